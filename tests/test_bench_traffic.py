"""Host logic of bench.py: the committed counter record is reported as the
traffic figure only for the launch configuration and the kernel sources it
was taken on (a changed source, tile shape, reordering period or warm-up
length gives null); a secondary leg that fails is reported in the line and
its resources are released."""
import glob
import json
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.traffic.json")))
HEADLINE = os.path.join(ROOT, "profiles", "k_particles_fp32_8192x2048_ppc64_order3.traffic.json")


def _record(path=HEADLINE):
    with open(path) as f:
        return json.load(f)


def _sources_hash(root, rec):
    import hashlib
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(root, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


@pytest.mark.parametrize("path", RECORDS, ids=os.path.basename)
def test_record_matches_its_configuration(path):
    rec = _record(path)
    cfg = rec["config"]
    r, src = bench.measured_traffic(cfg["precision"], tuple(cfg["tile"]), cfg["tile_split"],
                                    cfg["order"], cfg["particles"], cfg.get("sort_every", 0),
                                    cfg.get("warmup", 0))
    if _sources_hash(ROOT, rec) == rec["sources_sha256"]:
        assert r["traffic_bytes"] == rec["traffic_bytes"] and src.endswith(".traffic.json")
    else:
        # the kernel changed since the counters were taken: no figure
        assert (r, src) == (None, None)
    # traffic within a few percent of the algorithmic bytes (nothing re-read)
    assert 1.0 <= rec["traffic_bytes"] / rec["algorithmic_bytes"] <= 1.1


def test_other_configurations_get_no_figure():
    rec = _record()
    cfg = rec["config"]
    args = [cfg["precision"], tuple(cfg["tile"]), cfg["tile_split"], cfg["order"],
            cfg["particles"], cfg.get("sort_every", 0), cfg.get("warmup", 0)]
    for k, v in ((1, (16, 16)), (2, cfg["tile_split"] + 1), (5, cfg.get("sort_every", 0) + 1),
                 (6, cfg.get("warmup", 0) + 1), (0, "fp64")):
        a = list(args)
        a[k] = v
        assert bench.measured_traffic(*a) == (None, None), k


def test_changed_source_gets_no_figure(tmp_path, monkeypatch):
    rec = _record()
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    for src in rec["sources"]:
        dst = root / src
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), dst)
    # a record taken on exactly these sources
    rec = dict(rec, sources_sha256=_sources_hash(str(root), rec))
    with open(root / "profiles" / os.path.basename(HEADLINE), "w") as f:
        json.dump(rec, f)
    monkeypatch.setattr(bench, "ROOT", str(root))
    cfg = rec["config"]
    args = (cfg["precision"], tuple(cfg["tile"]), cfg["tile_split"], cfg["order"],
            cfg["particles"], cfg.get("sort_every", 0), cfg.get("warmup", 0))
    assert bench.measured_traffic(*args)[0]["traffic_bytes"] == rec["traffic_bytes"]
    with open(root / rec["sources"][0], "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic(*args) == (None, None)


def test_headline_record_is_current_and_gives_ceilings():
    """The headline configuration's record is taken on the committed kernel
    sources, and the ceilings follow from its counts: the VALU issue time of
    the counted instructions and the LDS pipe's active fraction."""
    rec = _record()
    if _sources_hash(ROOT, rec) != rec["sources_sha256"]:
        pytest.skip("the particle kernel changed since its counters were taken")
    cfg = rec["config"]
    assert (tuple(cfg["tile"]), cfg["tile_split"], cfg["sort_every"]) == \
        (bench.HEADLINE_TILE, bench.HEADLINE_SPLIT, bench.HEADLINE_SORT)
    c = bench.ceilings(rec, cfg["particles"], 60.0)
    waves = cfg["particles"] / 64
    valu_ms = waves * rec["valu_instructions_per_wavefront_of_64_particles"] * 4 / (1024 * 2.4e9)
    assert abs(c["valu_issue"]["ms"] - 1e3 * valu_ms) < 1e-9
    assert abs(c["valu_issue"]["frac"] - 1e3 * valu_ms / 60.0) < 1e-12
    assert 0.0 < c["lds"]["active_fraction_counted"] <= 1.0
    assert bench.ceilings(None, cfg["particles"], 60.0) is None


def test_failed_leg_is_reported_not_raised():
    class Held:
        alive = 0

        def __init__(self):
            Held.alive += 1

        def __del__(self):
            Held.alive -= 1

    def failing():
        ctx = Held()   # stands for a context holding a workspace
        raise RuntimeError(f"batched pic_step returned PIC_E_CAPACITY ({ctx is not None})")

    out = bench.run_leg("batched sweep", failing)
    assert out == {"error": "RuntimeError: batched pic_step returned PIC_E_CAPACITY (True)"}
    assert Held.alive == 0
    assert bench.run_leg("network rate", lambda: {"ms": 1.0}) == {"ms": 1.0}
