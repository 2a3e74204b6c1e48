"""Host logic of the launch-variant autotuner: cache keys, the choice of the fastest
variant and the JSON cache round trip (no GPU)."""
import json

import pytest

from paper_2212_10733_amd import autotune


def test_key_and_best(tmp_path):
    assert autotune.key("gfx950:sramecc+:xnack-", 33, 37, "f32", True) == "gfx950|33x37|f32|uniform"
    assert autotune.key("gfx950", 39, 39, "f64", False) == "gfx950|39x39|f64|vol"
    assert autotune.best({"auto": 2.0, "wave": 1.5, "block_256x6": 3.0}) == "wave"
    assert autotune.best({"auto": 1.0, "wave": 1.0}) == "auto"          # ties keep the earlier one
    path = str(tmp_path / "c.json")
    assert autotune.load(path) == {}
    c = {"gfx950|39x39|f32|uniform": {"variant": "wave_fixed", "ms": {"auto": 1.0, "wave_fixed": 1.0}}}
    autotune.save(path, c)
    assert autotune.load(path) == c
    with open(path, "w") as f:
        json.dump([1, 2], f)
    with pytest.raises(ValueError):
        autotune.load(path)
