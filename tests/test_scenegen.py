"""Seeded workload generators: determinism and the sizes the workloads state."""
import numpy as np

import scenegen as sg


def test_scenes_are_deterministic_and_sized():
    assert sg.make_toy().digest() == sg.make_toy().digest()
    u1, u2 = sg.make_urban(0), sg.make_urban(0)
    assert u1.digest() == u2.digest() and u1.nt == 770
    assert sg.make_urban(1).digest() != u1.digest()
    assert sg.make_toy().nt == 14
    h = np.asarray([r[2] for r in u1.roofs])
    assert 10.0 <= h.min() and h.max() <= 60.0
    assert set(np.unique(u1.tri_mat)) == {0, 1}


def test_city_scene_size_small_variant():
    c = sg.make_city(0, blocks=6)
    # per building 4n - 4 triangles with n in 5..8, plus 2 ground triangles
    nb = 6 * 6 * 4
    assert 16 * nb + 2 <= c.nt <= 28 * nb + 2
    assert set(np.unique(c.tri_mat)) <= {0, 1, 2}


def test_workload_devices():
    w = sg.toy_workload()
    assert len(w.rx) == 16 and w.num_rays == 100_000 and w.max_depth == 1
    for r in w.rx:
        x, y, z = r.pos
        assert z == 1.5 and not (29 <= x <= 51 and -6 <= y <= 6)
    u = sg.urban_workload()
    assert u.num_rays == 10_000_000 and u.max_depth == 3 and u.grid.nx == 400
    d = sg.diff_workload()
    assert len(d.rx) == 256 and d.tx[0].pattern == sg.PATTERN_TR38901
