"""The workload configuration files and the generators that read them (no GPU)."""

import json
from pathlib import Path

import pytest

import synth

CFG_DIR = Path(synth.__file__).with_name("configs")


@pytest.mark.parametrize("c", range(5))
def test_each_configuration_loads_and_is_a_copy(c):
    cfg = synth.config(c)
    assert cfg == json.loads((CFG_DIR / f"cfg{c}.json").read_text())
    cfg["name"] = "changed"
    assert synth.config(c)["name"] != "changed"


def test_missing_configuration_is_an_error():
    with pytest.raises(ValueError):
        synth.config(5)


@pytest.mark.parametrize("c", [0, 1, 4])
def test_frame_workloads_take_their_shapes_from_the_files(c):
    cfg = synth.config(c)
    side = 32 if c != 0 else None
    w = synth.workload(c, texture_side=side)
    fr = cfg["frame"]
    assert (w["n"], w["k"], w["width"], w["height"]) == (cfg["n"], cfg["k"], fr["width"], fr["height"])
    p = w["paths"]
    assert (p.spp, p.l_min, p.l_max, p.seed) == (fr["spp"], *fr["path_length"], cfg["path_seed"])
    lt = cfg["lights"]
    assert w["illum"].shape == (lt["planck"] + lt["narrow"], cfg["n"])
    assert w["n_tex"] == (cfg["reflectances"] if c == 0 else side * side)


def test_serving_mix_follows_its_configuration():
    from paper_2602_18741_amd.serve import make_requests
    cfg = synth.config(3)
    reqs = make_requests(rate=100.0, count=400, n_assets=cfg["assets"], seed=9)
    assert {(r.width, r.height) for r in reqs} == {tuple(x) for x in cfg["resolutions"]}
    assert {r.spp for r in reqs} == set(cfg["spp"])
    assert {(r.l_min, r.l_max) for r in reqs} == {tuple(cfg["path_length"])}
    assert all(0 <= r.asset < cfg["assets"] for r in reqs)
