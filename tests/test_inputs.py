"""Input generators: determinism, the paper's stated acquisition geometry, workload shapes."""

import json
import os

import numpy as np

import bos_inputs as bi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_geometry_fixture():
    with open(os.path.join(GOLDEN, "paper_workload.json")) as f:
        g = json.load(f)
    sc = bi.scene_paper_geometry()
    assert list(sc.cam_pos) == g["camera_position_m"]["value"]
    assert list(sc.proj_pos) == g["projector_position_m"]["value"]
    assert list(sc.cam_fwd) == g["view_direction"]["value"] == list(sc.proj_fwd)
    assert [sc.width, sc.height] == g["sensor_resolution"]["value"]
    assert list(sc.dims) == g["reconstruction_grid"]["value"]
    # projector offset +1 m in x from the camera, as in the paper's setup
    assert np.allclose(np.subtract(sc.proj_pos, sc.cam_pos), [1.0, 0.0, 0.0])


def test_seeded_fields_are_deterministic_and_hot():
    a = bi.plumes_room(3)
    b = bi.plumes_room(3)
    assert a == b and 4 <= len(a.plumes) <= 8
    sc = bi.scene_room((24, 20, 16), 8, 8)
    T = bi.temperature_grid(a, sc.box_lo, sc.box_hi, sc.dims)
    assert T.shape == (16, 20, 24) and T.dtype == np.float64
    assert T.min() >= 293.0 and T.max() <= 293.0 + 0.5 * 3.0 + 8.0 * len(a.plumes)
    for p in a.plumes:
        assert 0.1 <= p.sigma <= 0.5 and 1.0 <= p.amplitude <= 8.0


def test_patterns_and_subsets():
    d = bi.binary_dots(11)
    assert d.shape == (256, 256) and set(np.unique(d)) <= {0.0, 1.0}
    assert abs(d.mean() - 0.3) < 0.01
    n = bi.blurred_noise(12, (64, 64))
    assert n.shape == (64, 64) and 0.0 <= n.min() and n.max() <= 1.0
    ids = bi.pixel_subset(1000, 100, 15)
    assert len(np.unique(ids)) == 100 and ids.dtype == np.int32
    st = bi.strided_tiles(20, 12, 8, 2)
    assert len(np.unique(st)) == len(st) and st.max() < 240


def test_batch_recipe():
    scenes = bi.scenes_batch(4)
    for sc, spec in scenes:
        assert all(48 <= n <= 192 for n in sc.dims)
        assert 128 <= sc.width <= 1024 and 128 <= sc.height <= 1024
        assert sc.max_steps % 16 == 0 and sc.max_steps * sc.step > 1.1 * 6.4
        assert 4 <= len(spec.plumes) <= 8
    # deterministic per seed
    assert bi.scenes_batch(2)[1][1] == bi.scenes_batch(2)[1][1]


def test_network_inputs_seeded_and_shaped():
    import bos_inputs as bi

    lo, hi = (0.0, 0.0, 0.0), (4.0, 4.0, 3.0)
    th = bi.mlp_params(64, 4, 7, out_scale=0.3, bias_std=0.05)
    assert th.size == 3 * 64 + 64 + 3 * (64 * 64 + 64) + 64 * 5 + 5
    assert np.array_equal(th, bi.mlp_params(64, 4, 7, out_scale=0.3, bias_std=0.05))
    assert not np.array_equal(th, bi.mlp_params(64, 4, 8, out_scale=0.3, bias_std=0.05))
    # Glorot bound per layer, the last one scaled
    o = 0
    shapes = bi.mlp_param_shapes(64, 4)
    for i, (fi, fo) in enumerate(shapes):
        lim = np.sqrt(6.0 / (fi + fo)) * (0.3 if i == len(shapes) - 1 else 1.0)
        W = th[o:o + fi * fo]
        assert np.abs(W).max() <= lim and np.abs(W).max() > 0.5 * lim
        o += fi * fo + fo
    pb = bi.inlet_points(1000, lo, hi, 5)
    assert np.all(pb[:, 0] == lo[0]) and np.all((pb[:, 1:] >= lo[1:]) & (pb[:, 1:] <= hi[1:]))
    pc = bi.collocation_points(1000, lo, hi, 6)
    assert np.all((pc >= lo) & (pc <= hi)) and np.array_equal(pc, bi.collocation_points(1000, lo, hi, 6))
