"""Shape, determinism and recipe checks of the synthetic input generators."""
import numpy as np

import synth


def test_room_recipe():
    r = synth.room()
    txyz, tcov = r["target"]
    sxyz, scov = r["source"]
    assert txyz.shape == (3, 5000) and tcov.shape == (6, 5000)
    assert txyz.dtype == np.float32 and tcov.dtype == np.float32
    # every target point sits on a face of the 10 x 8 x 3 m room, up to the 1 cm noise
    half = np.array([5.0, 4.0, 1.5])[:, None]
    face_dist = np.min(np.abs(np.abs(txyz) - half), axis=0)
    assert face_dist.max() < 0.06
    # covariance 0.01 * (I - 0.999 n n^T): trace 0.01 * 2.001, smallest eigenvalue 1e-5
    tr = tcov[0] + tcov[3] + tcov[5]
    np.testing.assert_allclose(tr, 0.02001, rtol=1e-5)
    G = r["G"]
    ang = np.degrees(np.arccos(np.clip((np.trace(G[:3, :3]) - 1) / 2, -1, 1)))
    assert ang <= 5.0 and np.linalg.norm(G[:3, 3]) <= 0.3
    assert sxyz.shape == (3, 5000) and scov.shape == (6, 5000)


def test_room_deterministic():
    a, b = synth.room(), synth.room()
    np.testing.assert_array_equal(a["target"][0], b["target"][0])
    np.testing.assert_array_equal(a["source"][1], b["source"][1])
    c = synth.room(item=1)
    assert not np.array_equal(a["target"][0], c["target"][0])


def test_urban_sizes():
    u = synth.urban(0)
    n_s = u["source"][0].shape[1]
    assert 15_000 < n_s < 25_000
    assert len(u["targets"]) == 8
    for xyz, cov in u["targets"]:
        assert 45_000 < xyz.shape[1] < 70_000
        assert cov.shape == (6, xyz.shape[1])
    assert len(u["factors"]) == 24
    # FP32 points within the 80 m range of the sensor (plus noise)
    r = np.linalg.norm(u["source"][0].astype(np.float64), axis=0)
    assert r.max() < 80.5


def test_loop_path_closed():
    p0 = synth.loop_point(0.0)
    p1 = synth.loop_point(2000.0)
    assert abs(p0[0] - p1[0]) < 1e-6 and abs(p0[1] - p1[1]) < 1e-6
