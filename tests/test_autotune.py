"""Host logic of the autotuner's cache (no GPU): keys by workload,
architecture and precision; a missing or unreadable cache reads as absent."""
import json

import paper_2505_00715_amd as g
from paper_2505_00715_amd import autotune


def test_cache_roundtrip_and_keys(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "device_arch", lambda device=0: "gfx950")
    path = str(tmp_path / "t" / "tuning.json")
    assert autotune.load("sphere20480", g.C64, path) is None
    p = {"aca_waves": 2, "aca3d_waves": [4, 4, 4, 4], "aca3d_stack_slices": 8, "product_graph": 1}
    autotune.save("sphere20480", g.C64, p, path)
    assert autotune.load("sphere20480", g.C64, path) == p
    assert autotune.load("sphere20480", g.C128, path) is None
    assert autotune.load("housing40k", g.C64, path) is None
    monkeypatch.setattr(autotune, "device_arch", lambda device=0: "gfx942")
    assert autotune.load("sphere20480", g.C64, path) is None
    with open(path) as fh:
        assert "sphere20480|gfx950|c64" in json.load(fh)


def test_unreadable_cache_is_absent(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "device_arch", lambda device=0: "gfx950")
    path = tmp_path / "tuning.json"
    path.write_text("{not json")
    assert autotune.load("sphere20480", g.C64, str(path)) is None


def test_apply_sets_every_parameter():
    ctx = g.Context(-1)
    autotune.apply(ctx, {"aca_waves": 4, "aca3d_waves": [1, 2, 4, 8], "aca3d_stack_slices": 16,
                         "product_graph": 0})
    t = ctx.get_tuning()
    assert (t.aca_waves, list(t.aca3d_waves), t.aca3d_stack_slices, t.product_graph) == \
        (4, [1, 2, 4, 8], 16, 0)


def test_product_graph_choice_prefers_the_graph():
    assert autotune.choose_product_graph({0: 1.00, 1: 1.02}) == 1
    assert autotune.choose_product_graph({0: 1.02, 1: 1.00}) == 1
    assert autotune.choose_product_graph({0: 0.90, 1: 1.00}) == 0
