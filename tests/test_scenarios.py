"""The seeded input recipes: sizes, determinism and the shapes they promise."""
import numpy as np

from paper_2008_11578_amd import scenarios


def test_c1_shape_and_determinism():
    a = scenarios.c1_plain()
    b = scenarios.c1_plain()
    assert a.n == 256 and a.params.max_neighbors == 10 and a.steps == 20
    for k, v in a.arrays().items():
        np.testing.assert_array_equal(v, getattr(b, k))
        assert v.flags.c_contiguous
    assert a.px.dtype == np.float32 and a.cls.dtype == np.uint8
    assert (a.px >= 0).all() and (a.px <= 30).all()


def test_c2_mixed_classes():
    sc = scenarios.c2_mixed()
    assert sc.n == 66560
    assert int(sc.cls.sum()) == 1024
    veh = sc.cls == 1
    assert np.allclose(sc.radius[veh], 1.5) and np.allclose(sc.max_speed[veh], 6.0)
    # vehicle goals lie on the square's perimeter
    gx, gy = sc.pref_x[veh].astype(float), sc.pref_y[veh].astype(float)
    edge = np.minimum.reduce([gx, gy, 500 - gx, 500 - gy])
    assert np.abs(edge).max() < 1e-3


def test_crossing_lattice_no_overlap_and_groups():
    sc = scenarios.c3_crossing(side_count=128)   # same recipe, smaller
    assert sc.n == 128 * 128
    x = sc.px.astype(float)
    y = sc.py.astype(float)
    side = 700.0 * 128 / 1024
    spacing = side / 128
    # jitter 0.04 m per axis keeps neighbours at least spacing - 0.08 apart (> 2r)
    assert spacing - 0.08 > 0.6
    # goals are mirror images across the centre line parallel to each group's side
    gx, gy = sc.pref_x.astype(float), sc.pref_y.astype(float)
    horiz = np.abs(x - side / 2) > np.abs(y - side / 2)
    np.testing.assert_allclose(gx[horiz], side - x[horiz], atol=1e-4)
    np.testing.assert_allclose(gy[~horiz], side - y[~horiz], atol=1e-4)
    frac = horiz.mean()
    assert 0.45 < frac < 0.55


def test_c4_scene_offsets():
    sc = scenarios.c4_batched(n_scenes=16)
    off = sc.scene_off
    assert off[0] == 0 and off[-1] == sc.n and (np.diff(off) >= 64).all()
    assert len(sc.scene_params) == 16


def test_c5_rollout_targets():
    sc = scenarios.c5_rollout(n=512)
    assert sc.params.pref_is_goal == 0
    sp = np.hypot(sc.pref_x, sc.pref_y)
    np.testing.assert_allclose(sp, 1.4, rtol=1e-6)
    assert (sp < sc.max_speed).all()
    assert sc.target_x is not None and sc.target_x.shape == (512,)


def test_c2_vehicle_share_same_geometry():
    base = scenarios.c2_vehicle_share(0.0)
    half = scenarios.c2_vehicle_share(0.5)
    assert base.n == half.n == 66560
    assert int(base.cls.sum()) == 0 and int(half.cls.sum()) == 33280
    # vehicles are the last agents; the pedestrians' positions do not depend on the share
    np.testing.assert_array_equal(base.px[:1000], half.px[:1000])
