"""The ESDF oracle against what the paper and plain geometry fix (no GPU needed), and
plausible mistakes planted in copies of it, each caught by a pin."""
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import esdf
from tests import esdf_pins


@pytest.fixture(scope="module")
def esdf_lib():
    esdf.build()
    return esdf.load()


@pytest.mark.parametrize("pin", esdf_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(esdf_lib, pin):
    pin()


MUTATIONS = {
    "unit_steps": ("return E->v * sqrt((double)k);", "return E->v;"),
    "euclidean_squared_steps": ("return E->v * sqrt((double)k);", "return E->v * (double)k;"),
    "raise_keeps_distance": ("            x->d = (x->neg ? -1.0 : 1.0) * E->d_max;\n            x->parent = 13;\n",
                             "            x->parent = 13;\n"),
    "child_test_reversed": ("if (!y->fixed && y->parent == 26 - n)", "if (!y->fixed && y->parent == n)"),
    "band_overwritten": ("if (!y || !y->observed || y->fixed) continue;", "if (!y || !y->observed) continue;"),
    "parent_points_away": ("y->parent = (int8_t)(26 - n);      /* from y towards x */",
                           "y->parent = (int8_t)n;"),
    "new_free_voxel_alone": ("if (m != 13) insert_lower(E, neighbour_key(k, m));", "(void)m;"),
    "band_inclusive": ("if (-E->gamma < dt && dt < E->gamma) {", "if (-E->gamma <= dt && dt <= E->gamma) {"),
    "moved_band_voxel_not_raised": (
        "                x->parent = 13;\n                fifo_push(&E->raise, k);\n                insert_lower(E, k);",
        "                x->parent = 13;\n                insert_lower(E, k);"),
    "left_band_not_raised": ("            x->parent = 13;\n            fifo_push(&E->raise, k);\n        } else if",
                             "            x->parent = 13;\n        } else if"),
    "side_frozen": ("} else if (x->fixed || (x->observed && (dt < 0.0) != (x->neg != 0))) {",
                    "} else if (x->fixed) {"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(esdf_lib, name):
    old, new = MUTATIONS[name]
    src = open(esdf._SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    tmp = tempfile.mkdtemp(prefix="esdf_mut_")
    try:
        path = os.path.join(tmp, "esdf_oracle.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = os.path.join(tmp, "liboracle_esdf_mut.so")
        esdf.build(out=lib, src=path)
        caught = []
        for pin in esdf_pins.ALL_PINS:
            try:
                pin(lib)
            except AssertionError:
                caught.append(pin.__name__)
                break
        assert caught, f"planted mistake '{name}' passed every pin"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
