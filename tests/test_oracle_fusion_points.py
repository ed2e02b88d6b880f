"""The reference's fusion of listed lattice points (orc_fuse_points, Sec. 3.2.1) against its
fusion of the whole lattice, and the weight cap over a long sequence.

* Over three frames, the listed points hold exactly the values the whole-lattice fusion
  gives them (the same update, read and written through compact storage).
* The same frame fused 150 times: every updated point ends at weight 100 (the cap), and,
  the observation being the same every time, its tsdf and colour stay at the first
  frame's values (the running average of equal values) up to rounding.
"""
import numpy as np

import synth
from oracle import oracle as O


def _frames(n, W=96, H=72):
    scene = synth.scene_room(64)
    cams = synth.orbit_cameras(0, W, H, frames=list(range(0, 10 * n, 10)))
    return scene, [(c.as_dict(), *synth.render_frame(scene, c, noise_sigma_per_m2=2e-3, frame_index=k))
                   for k, c in enumerate(cams)]


def test_points_equal_whole_lattice():
    scene, fr = _frames(3)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    vol = O.new_volume(grid)
    rng = np.random.Generator(np.random.PCG64(8))
    N = int(np.prod(scene.dims))
    idx = np.sort(rng.choice(N, 4000, replace=False))
    pts = O.new_points(idx.size)
    for cam, d, c in fr:
        O.fuse(grid, vol, cam, d, c)
        O.fuse_points(grid, idx, pts, cam, d, c)
    assert (vol["weight"][idx] > 0).sum() > 200
    np.testing.assert_array_equal(pts["weight"], vol["weight"][idx])
    np.testing.assert_array_equal(pts["rgb_weight"], vol["rgb_weight"][idx])
    np.testing.assert_array_equal(pts["tsdf"], vol["tsdf"][idx])
    np.testing.assert_array_equal(pts["rgb"], vol["rgb"][:, idx])


def test_weight_cap_over_a_long_sequence():
    scene, fr = _frames(1)
    cam, d, c = fr[0]
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    N = int(np.prod(scene.dims))
    idx = np.arange(0, N, 7, dtype=np.int64)
    once = O.fuse_points(grid, idx, O.new_points(idx.size), cam, d, c)
    pts = O.new_points(idx.size)
    for _ in range(150):
        O.fuse_points(grid, idx, pts, cam, d, c)
    upd = once["weight"] > 0
    assert upd.sum() > 1000
    assert (pts["weight"][upd] == 100.0).all() and (pts["weight"][~upd] == 0.0).all()
    col = once["rgb_weight"] > 0
    assert (pts["rgb_weight"][col] == 100.0).all()
    assert np.abs(pts["tsdf"][upd] - once["tsdf"][upd]).max() < 1e-13
    assert np.abs(pts["rgb"][:, col] - once["rgb"][:, col]).max() < 1e-13
