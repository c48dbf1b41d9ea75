"""The autotuner's tile cache (BST_TUNE_CACHE) on the host: choices recorded
by one plan are read back by later plans of the same GEMM structure, other
structures keep their defaults, and malformed lines are skipped."""
import json

import pytest

from paper_2401_01921_amd import bst, workloads as wl


def _plan(chi, qmax, prec="fp64"):
    v = wl.gaussian_sector_dims(chi, qmax)
    T = {k: bst.Tensor(*s) for k, s in wl.heff_specs("1/2", v, v).items()}
    return T, bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], prec)


def _tiles(plan, prec):
    plan.set_precision(prec)
    return plan.tiles()


def test_record_requires_the_variable(monkeypatch):
    monkeypatch.delenv("BST_TUNE_CACHE", raising=False)
    _, p = _plan(128, 4)
    with pytest.raises(bst.BstError):
        p.record_tiles()


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("BST_TUNE_CACHE", str(path))
    _, a = _plan(512, 8)
    _, other0 = _plan(256, 6)
    default = {f: _tiles(a, f) for f in ("fp64", "bf16x3")}
    default_other = {f: _tiles(other0, f) for f in ("fp64", "bf16x3")}
    # a non-default choice in each form
    chosen = {}
    for f in ("fp64", "bf16x3"):
        n = a.tile_count(f)
        assert n >= 2
        for k in range(n):
            a.set_tile(f, k)
            if _tiles(a, f) != default[f]:
                break
        chosen[f] = _tiles(a, f)
        assert chosen[f] != default[f]
    a.record_tiles()
    entries = json.loads(path.read_text())
    assert len(entries) >= 2 and all(len(v) == 4 for v in entries.values())
    # a later plan of the same structure starts from the recorded choices
    _, b = _plan(512, 8)
    for f in ("fp64", "bf16x3"):
        assert _tiles(b, f) == chosen[f], f
    # another structure is unaffected
    _, c = _plan(256, 6)
    for f in ("fp64", "bf16x3"):
        assert _tiles(c, f) == default_other[f], f
    # recording a second structure keeps the first one's entries
    c.set_tile("fp64", 1)
    c.record_tiles()
    again = json.loads(path.read_text())
    assert set(entries) <= set(again) and len(again) > len(entries)
    # malformed lines are skipped, valid ones still apply
    path.write_text("garbage\n" + path.read_text() + "\n\"x\": [oops]\n")
    _, d = _plan(512, 8)
    assert _tiles(d, "fp64") == chosen["fp64"]


def test_fp64_variant_round_trip(tmp_path, monkeypatch):
    """The FP64 variant choice (float64 panels or per-block-pair kernels) is
    cached beside the tiles: an entry [1, 0, 0, 0] under the plan's variant
    key makes a later plan of the same structure start on the panels."""
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("BST_TUNE_CACHE", str(path))
    _, a = _plan(512, 8)
    blocks = _tiles(a, "fp64")
    a.record_tiles()
    entries = json.loads(path.read_text())
    variant = [k for k, v in entries.items() if v == [0, 0, 0, 0]]
    assert len(variant) == 1, entries
    entries[variant[0]] = [1, 0, 0, 0]
    path.write_text(json.dumps(entries))
    _, b = _plan(512, 8)
    panels = _tiles(b, "fp64")
    assert panels != blocks
    assert all("p" in t.split(":")[1] for t in panels.split(";") if t.startswith("gemm")), panels
