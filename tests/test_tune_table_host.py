"""The committed tuning table is consistent with the library it ships with:
each entry's tile index names the shape it records, that shape is the
fastest of the entry's timings and one the library runs for the entry's
kernel, and every 2D acoustic entry picks a two-steps-per-launch shape."""
import json

import pytest

import paper_2310_00236_amd as hw
from paper_2310_00236_amd import tuning

with open(tuning.TABLE) as f:
    TABLE = json.load(f)


@pytest.mark.parametrize("key", sorted(TABLE))
def test_entry_is_consistent(key):
    arch, physics, order, storage, comp, cells = key.split("/")
    assert arch == tuning.ARCH
    e = TABLE[key]
    shapes = hw.tiles(physics)
    shape = shapes[e["tile"]]
    assert list(shape) == list(e["shape"])
    times = e["ms_per_step"]
    assert hw.tile_label(shape) == min(times, key=times.get)
    assert set(times) <= {hw.tile_label(s) for s in shapes}
    pb = hw.Problem(physics, 8, 8, 8 if physics == "elastic3d" else 1, int(order[1:]),
                    storage, comp, 1.0, 0.01, 0, 0)
    assert tuning.supported(pb, shape)
    if physics == "acoustic2d":
        assert shape[2] == 2, "a two-step shape"


def test_lookup_falls_back_to_the_nearest_bucket():
    """A size with no entry of its own takes the nearest measured bucket's
    shape (8192^2 -> the 4096^2 entry)."""
    assert tuning.key("acoustic2d", 4, "f16", "twosum", 8192, 8192) not in TABLE
    near = TABLE[tuning.key("acoustic2d", 4, "f16", "twosum", 4096, 4096)]["tile"]
    assert tuning.best_tile("acoustic2d", 4, "f16", "twosum", 8192, 8192) == near
