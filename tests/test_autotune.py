"""Host logic of the tile autotuner: size classes, representatives and table lookup."""
import math

import pytest

from paper_2406_09423_amd import autotune


def test_classes_are_monotone_and_cover_the_batch():
    import synth
    shapes, _ = synth.batch_shapes(0)
    seen = set()
    for s in shapes:
        seen.add(autotune.size_class(s))
    assert all(c.split(":")[0] in ("2d", "3d") for c in seen)
    for ndim in (2, 3):
        prev = -1
        for side in (4, 16, 64, 128, 512, 2048, 8192) if ndim == 2 else (8, 16, 32, 64, 128, 192, 256, 512):
            k = int(autotune.size_class((side,) * ndim).split(":")[1])
            assert k >= prev
            prev = k
        assert prev == autotune.n_classes(ndim) - 1


@pytest.mark.parametrize("ndim", [2, 3])
def test_representatives_fall_in_their_class(ndim):
    for k in range(autotune.n_classes(ndim)):
        cls = f"{ndim}d:{k}"
        shape = autotune.representative(cls)
        assert len(shape) == ndim
        assert autotune.size_class(shape) == cls, (cls, shape, math.prod(shape))


def test_lookup_from_a_table():
    table = {"classes": {"2d:2": {"variant": 2}, "3d:1": {"variant": 3}}}
    assert autotune.tile_for((300, 300), table) == 2        # 90,000 vertices: class 2
    assert autotune.tile_for((40, 40, 40), table) == 3      # 64,000: class 1
    assert autotune.tile_for((10, 10), table) == 0          # untuned class: default tile
    assert autotune.tiles_for([(300, 300), (10, 10)], table) == [2, 0]
    assert autotune.tile_for((300, 300), {}) == 0


def test_stored_table_is_valid():
    table = autotune.load_table()
    if table is None:
        pytest.skip("no tuned table stored")
    limits = {2: 2, 3: 4}
    for cls, entry in table["classes"].items():
        ndim = int(cls[0])
        assert 1 <= entry["variant"] <= limits[ndim]
        assert str(entry["variant"]) in entry["us_per_launch"]
        assert entry["us_per_launch"][str(entry["variant"])] == min(entry["us_per_launch"].values())
