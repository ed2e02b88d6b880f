"""Pins of the reference's voxel-block allocation and of fusion into allocated blocks
(Sec. 3.2.1, "SDF fusion": the SDF lives in a hash table of voxel blocks, following
InfiniTAM).

* The binary32 block decisions agree with the definition evaluated in binary64
  (the ray point at depth d + k voxel, floor of its block coordinate) for every
  sample farther than 1e-4 of a block edge from a block face; samples nearer a face
  may land in either neighbour.
* A fronto-parallel plane at constant depth allocates, in every block layer the band
  reaches, a full rectangle of blocks whose bounds are those of the frustum's
  cross-section (pixel spacing is far below the block edge, so no block between the
  extremes is missed); the layers are those of the band's depths.
* Accumulation: the blocks of two frames are the union of each frame's blocks; no
  depth, no block; one pixel gives a chain of face-, edge- or corner-adjacent blocks.
* Fusion with a block mask: with every block allocated it is the unmasked fusion, bit
  for bit; otherwise the points of unallocated blocks keep tsdf 1, weight 0, colour 0
  and the others hold exactly the unmasked result.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from synth.scene import small_camera

BLOCK = 8


def _samples64(grid, cam, depth, block=BLOCK):
    """Block coordinate (binary64) of every sample of the definition, and whether it lies
    within 1e-4 of a block face."""
    H, W = depth.shape
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    K = int(np.ceil(float(np.float32(grid.trunc)) / float(np.float32(grid.voxel))))
    jj, ii = np.nonzero(depth > 0)
    d = depth[jj, ii].astype(np.float64)
    xn = (ii - float(np.float32(cam["cx"]))) / float(np.float32(cam["fx"]))
    yn = (jj - float(np.float32(cam["cy"]))) / float(np.float32(cam["fy"]))
    out, near = [], []
    bsz = float(np.float32(grid.voxel)) * block
    org = np.array([grid.origin[k] for k in range(3)], np.float64)
    for k in range(-K, K + 1):
        z = d + k * float(np.float32(grid.voxel))
        ok = z > 0
        xc = np.stack([xn * z, yn * z, z])[:, ok]
        p = R.T @ (xc - t[:, None])
        r = (p - org[:, None]) / bsz
        out.append(np.floor(r).astype(np.int64))
        near.append((np.abs(r - np.round(r)) < 1e-4).any(axis=0))
    return np.concatenate(out, axis=1), np.concatenate(near)


def _set_of(mask):
    bz, by, bx = np.nonzero(mask)
    return set(zip(bx.tolist(), by.tolist(), bz.tolist()))


def _room_frame(W=160, H=120, frame=3):
    scene = synth.scene_room()
    cam = synth.orbit_cameras(0, W, H, frames=[frame])[0]
    d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=frame)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    return scene, cam.as_dict(), d, c, grid


def test_binary32_blocks_agree_with_the_binary64_definition():
    scene, cam, d, c, grid = _room_frame()
    mask = O.alloc_blocks(grid, cam, d)
    got = _set_of(mask)
    b64, near = _samples64(grid, cam, d)
    nb = np.array(O.block_grid(grid))[:, None]
    inside = ((b64 >= 0) & (b64 < nb)).all(axis=0)
    firm = {tuple(x) for x in b64[:, inside & ~near].T.tolist()}
    loose = {tuple(x) for x in b64[:, inside].T.tolist()}
    assert len(firm) > 300
    assert firm <= got                       # every block a firm sample reaches is allocated
    extra = got - loose                      # blocks only a near-face sample reaches
    for b in extra:                          # ... must be a face neighbour of a reached block
        assert any(tuple(np.add(b, o)) in loose for o in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                                          (0, 0, 1), (0, 0, -1)))
    missing = loose - got
    assert len(missing) <= (near & inside).sum()
    print(f"blocks {len(got)}, firm {len(firm)}, near-face samples {(near & inside).sum()}, "
          f"flipped blocks {len(extra) + len(missing)}")


@pytest.mark.parametrize("D", [0.7, 1.13])
def test_fronto_parallel_plane_allocates_rectangles(D):
    W, H, f = 64, 48, 60.0
    cam = {"width": W, "height": H, "fx": f, "fy": f, "cx": W / 2 - 0.5, "cy": H / 2 - 0.5,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    grid = O.make_grid((128, 128, 128), (-1.28, -1.28, 0.0), 0.02, 0.08)
    depth = np.full((H, W), D, np.float32)
    mask = O.alloc_blocks(grid, cam, depth)
    bsz = 0.16
    zs = D + 0.02 * np.arange(-4, 5)
    layers = sorted({int(np.floor(z / bsz)) for z in zs})
    assert sorted(set(np.nonzero(mask)[0].tolist())) == layers
    for L in layers:
        zl = zs[np.floor(zs / bsz) == L]
        xs = np.concatenate([(np.array([0, W - 1]) - cam["cx"]) / f * z for z in zl])
        ys = np.concatenate([(np.array([0, H - 1]) - cam["cy"]) / f * z for z in zl])
        bx = np.floor((xs + 1.28) / bsz).astype(int)
        by = np.floor((ys + 1.28) / bsz).astype(int)
        want = np.zeros_like(mask[L])
        want[by.min():by.max() + 1, bx.min():bx.max() + 1] = 1
        np.testing.assert_array_equal(mask[L], want)


def test_allocation_accumulates_and_chains():
    scene, cam, d, c, grid = _room_frame(frame=3)
    _, cam2, d2, _, _ = _room_frame(frame=40)
    a = O.alloc_blocks(grid, cam, d)
    b = O.alloc_blocks(grid, cam2, d2)
    both = O.alloc_blocks(grid, cam2, d2, mask=a.copy())
    np.testing.assert_array_equal(both, a | b)
    assert not O.alloc_blocks(grid, cam, np.zeros_like(d)).any()
    one = np.zeros_like(d)
    one[60, 80] = d[60, 80]
    blocks = sorted(_set_of(O.alloc_blocks(grid, cam, one)))
    assert 1 <= len(blocks) <= 4
    # consecutive samples are one voxel apart, far below the block edge: the blocks form a chain
    left = set(blocks[1:])
    seen = [blocks[0]]
    while left:
        nxt = [b for b in left if any(max(abs(np.subtract(b, s))) <= 1 for s in seen)]
        assert nxt, (blocks, seen)
        for b in nxt:
            left.discard(b)
            seen.append(b)


def test_masked_fusion():
    w = synth.workload_small(M=10)
    sc, cam = w["scene"], w["cam"].as_dict()
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    dense = O.fuse(grid, O.new_volume(grid), cam, w["depth"], w["rgb"])
    full = np.ones(O.block_grid(grid)[::-1], np.uint8)
    allm = O.fuse(grid, O.new_volume(grid), cam, w["depth"], w["rgb"], block_mask=full)
    for k in dense:
        np.testing.assert_array_equal(allm[k], dense[k])
    mask = O.alloc_blocks(grid, cam, w["depth"])
    assert 0 < mask.sum() < mask.size
    hv = O.fuse(grid, O.new_volume(grid), cam, w["depth"], w["rgb"], block_mask=mask)
    n = sc.dims
    zz, yy, xx = np.meshgrid(*(np.arange(k) for k in n[::-1]), indexing="ij")
    inb = mask[zz // BLOCK, yy // BLOCK, xx // BLOCK].astype(bool).reshape(-1)
    np.testing.assert_array_equal(hv["tsdf"][inb], dense["tsdf"][inb])
    np.testing.assert_array_equal(hv["weight"][inb], dense["weight"][inb])
    np.testing.assert_array_equal(hv["rgb"][:, inb], dense["rgb"][:, inb])
    assert (hv["tsdf"][~inb] == 1).all() and (hv["weight"][~inb] == 0).all() and (hv["rgb"][:, ~inb] == 0).all()
    # the band around the surface is allocated: every updated point of the band is in a block
    band = (dense["rgb_weight"] > 0)
    assert inb[band].mean() > 0.95
