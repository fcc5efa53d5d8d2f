"""The launch table of the autotuner (klst_tune_save / klst_tune_load /
klst_tune_clear): text round trip and refusal of malformed entries.  CPU only
(no device needed; klst_autotune itself is exercised by the GPU tests)."""
import pytest

klst = pytest.importorskip("paper_2607_27440_amd.klst")


def test_table_round_trip(tmp_path):
    klst.tune_clear()
    src = tmp_path / "in.txt"
    src.write_text("# comment\n96 1464 1 0 1 1 5 8\n96 1464 64 0 6 4 0 0\n24 16 1 1 8 0 1 16\n")
    klst.tune_load(str(src))
    out = tmp_path / "out.txt"
    klst.tune_save(str(out))
    rows = sorted(tuple(int(v) for v in ln.split()) for ln in out.read_text().splitlines()
                  if ln and not ln.startswith("#"))
    assert rows == sorted([(96, 1464, 1, 0, 1, 1, 5, 8), (96, 1464, 64, 0, 6, 4, 0, 0), (24, 16, 1, 1, 8, 0, 1, 16)])
    klst.tune_clear()
    klst.tune_save(str(out))
    assert [ln for ln in out.read_text().splitlines() if ln and not ln.startswith("#")] == []


def test_table_refuses_malformed_lines(tmp_path):
    klst.tune_clear()
    bad = tmp_path / "bad.txt"
    bad.write_text("96 1464 1 0 1 1 5\n")
    with pytest.raises(klst.KlstError):
        klst.tune_load(str(bad))
    with pytest.raises(klst.KlstError):
        klst.tune_load(str(tmp_path / "missing.txt"))
    klst.tune_clear()
