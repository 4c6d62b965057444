"""The sketch launch-shape table (smp_tune_*): its JSON file round trip and
lookups through the C-ABI, without a GPU (the table and its file are host
code; the timing itself, smp_tune_sketch, is tested in test_gpu_tune.py)."""

import json

import pytest


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


def _entry(prec, k, n1, n2, rows, cap, splits, ms=0.5, srht=0):
    return {"prec": prec, "srht": srht, "k": k, "n1": n1, "n2": n2, "rows": rows, "cap": cap, "splits": splits,
            "ms": ms}


def _write(path, entries, version=1, fmt="smp-sketch-tuning"):
    path.write_text(json.dumps({"format": fmt, "version": version, "entries": entries}, indent=1))


def test_load_lookup_save_clear(api, tmp_path):
    api.smp_tune_clear()
    bf = api.make_params(10_000, 300, 200, 400, 5, prec=api.SMP_PREC_BF16)
    ab = api.make_params(10_000, 300, 300, 400, 5, prec=api.SMP_PREC_BF16, b_is_a=True)
    f32 = api.make_params(10_000, 300, 200, 64, 5)
    assert api.smp_tune_lookup(bf) == (0, 0)
    # rows per launch: d itself here (d is below one stored-Pi window)
    _write(tmp_path / "t.json", [_entry(1, 400, 300, 200, 10_000, 13, 6), _entry(1, 400, 300, 0, 10_000, 16, 3),
                                 _entry(0, 64, 300, 200, 10_000, 0, 2)])
    api.smp_tune_load(tmp_path / "t.json")
    assert api.smp_tune_lookup(bf) == (13, 6)
    assert api.smp_tune_lookup(ab) == (16, 3)          # B = A is its own shape (n2 = 0)
    assert api.smp_tune_lookup(f32) == (0, 2)
    assert api.smp_tune_lookup(api.make_params(10_001, 300, 200, 400, 5, prec=api.SMP_PREC_BF16)) == (0, 0)
    api.smp_tune_save(tmp_path / "out.json")
    doc = json.loads((tmp_path / "out.json").read_text())
    assert doc["format"] == "smp-sketch-tuning" and doc["version"] == 1
    got = {(e["prec"], e["k"], e["n2"]): (e["cap"], e["splits"]) for e in doc["entries"]}
    assert got == {(1, 400, 200): (13, 6), (1, 400, 0): (16, 3), (0, 64, 200): (0, 2)}
    api.smp_tune_clear()
    assert api.smp_tune_lookup(bf) == (0, 0)
    api.smp_tune_load(tmp_path / "out.json")           # the saved file loads back
    assert api.smp_tune_lookup(bf) == (13, 6)
    api.smp_tune_clear()


def test_bad_files_leave_the_table(api, tmp_path):
    api.smp_tune_clear()
    p = api.make_params(10_000, 300, 200, 400, 5, prec=api.SMP_PREC_BF16)
    _write(tmp_path / "good.json", [_entry(1, 400, 300, 200, 10_000, 16, 4)])
    api.smp_tune_load(tmp_path / "good.json")
    bad = {
        "version.json": dict(version=2, entries=[_entry(1, 400, 300, 200, 10_000, 13, 8)]),
        "format.json": dict(fmt="other", entries=[_entry(1, 400, 300, 200, 10_000, 13, 8)]),
        "missing.json": dict(entries=[{"prec": 1, "k": 400}]),
        "range.json": dict(entries=[_entry(5, 400, 300, 200, 10_000, 13, 8)]),
    }
    for name, kw in bad.items():
        _write(tmp_path / name, **kw)
        with pytest.raises(api.SmpError):
            api.smp_tune_load(tmp_path / name)
        assert api.smp_tune_lookup(p) == (16, 4), name
    with pytest.raises(api.SmpError):
        api.smp_tune_load(tmp_path / "does_not_exist.json")
    with pytest.raises(api.SmpError):
        api.smp_tune_save(tmp_path / "no_such_dir" / "x.json")
    api.smp_tune_clear()
