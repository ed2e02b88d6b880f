"""GPU parity of the voxel-block hash of the TSDF (Sec. 3.2.1, "SDF fusion" into a hash
table of voxel blocks) against the reference (orc_alloc_blocks, orc_fuse with the block
mask, orc_raycast of the masked lattice).

* Allocation: the set of allocated blocks equals the reference's, bit for bit (both
  decide each band point's block in binary32 with the same steps), after every frame.
* Fusion: at every lattice point of the allocated blocks, weights bit-exact, tsdf and
  colour within the binary32 bounds of the dense fusion tests (2e-5 after one frame,
  1e-4 after several); points outside them read tsdf 1, weight 0.
* Raycast: with the reference's binary32 lattice values loaded into the pool, the hit
  set equals the reference's and the depth is within 1e-4 of the largest depth; and the
  hashed raycast is bitwise the dense GPU raycast of the same lattice values, with and
  without the skipping of positive blocks and with and without the per-tile depth
  ranges that limit each ray's march.
* A pool that overflows sets its status bit, keeps every stored block consistent and is
  cleared by the reset; fusing the same frame again allocates nothing new.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, h, say, t

pytestmark = pytest.mark.gpu
B = 8


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    P.lib()
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.lib()
    return O


def _blocks(vol):
    n = min(vol.state()["allocated"], vol.capacity)
    k = vol.block_key[:n].cpu().numpy().view(np.uint64)
    m = np.uint64((1 << 21) - 1)
    return np.stack([(k & m), (k >> np.uint64(21)) & m, (k >> np.uint64(42)) & m]).astype(np.int64)


def _mask_set(mask):
    bz, by, bx = np.nonzero(mask)
    return set(zip(bx.tolist(), by.tolist(), bz.tolist()))


def _point_index(bc, dims):
    """Lattice index and pool index of every point of the pool blocks bc [3][n] (points
    inside the region only)."""
    nx, ny, nz = dims
    l = np.arange(B ** 3)
    lx, ly, lz = l % B, (l // B) % B, l // (B * B)
    x = (bc[0][:, None] * B + lx[None]).reshape(-1)
    y = (bc[1][:, None] * B + ly[None]).reshape(-1)
    z = (bc[2][:, None] * B + lz[None]).reshape(-1)
    pool = (np.arange(bc.shape[1])[:, None] * B ** 3 + l[None]).reshape(-1)
    ok = (x < nx) & (y < ny) & (z < nz)
    return (x + nx * (y + ny * z))[ok], pool[ok]


def _gather(vol, dims):
    """The hashed volume as a dense lattice (points of unallocated blocks: 1, 0, 0, 0)."""
    N = int(np.prod(dims))
    lat, pool = _point_index(_blocks(vol), dims)
    out = {"tsdf": np.ones(N, np.float32), "weight": np.zeros(N, np.float32), "rgb": np.zeros((3, N), np.float32),
           "rgb_weight": np.zeros(N, np.float32)}
    out["tsdf"][lat] = h(vol.tsdf)[pool]
    out["weight"][lat] = h(vol.weight)[pool]
    out["rgb"][:, lat] = h(vol.rgb)[:, pool]
    out["rgb_weight"][lat] = h(vol.rgb_weight)[pool]
    return out, lat


def _load(vol, dims, tsdf32, rgb32):
    """Writes lattice values into the pool blocks of the hashed volume."""
    lat, pool = _point_index(_blocks(vol), dims)
    pi = torch.as_tensor(pool, device=DEV)
    vol.tsdf[pi] = t(tsdf32.reshape(-1)[lat])
    vol.rgb[:, pi] = t(rgb32.reshape(3, -1)[:, lat])


def _check_volume(O, vol, grid, ref, mask, tol):
    dims = (grid.nx, grid.ny, grid.nz)
    assert _mask_set(mask) == {tuple(b) for b in _blocks(vol).T.tolist()}
    g, lat = _gather(vol, dims)
    np.testing.assert_array_equal(g["weight"], ref["weight"].astype(np.float32))
    np.testing.assert_array_equal(g["rgb_weight"], ref["rgb_weight"].astype(np.float32))
    assert np.abs(g["tsdf"] - ref["tsdf"]).max() <= tol
    assert np.abs(g["rgb"] - ref["rgb"]).max() <= tol
    return lat


def _raycast_checks(P, O, vol, grid, dims, cams, t32, c32, n_sample=None, z_near=0.2):
    """Hashed raycast of the reference's values: against the reference and, bitwise,
    against the dense GPU raycast of the same lattice."""
    _load(vol, dims, t32, c32)
    dense = P.Volume(dims, tuple(grid.origin), grid.voxel, grid.trunc, device=DEV)
    dense.tsdf.copy_(t(t32.reshape(-1)))
    dense.rgb.copy_(t(c32.reshape(3, -1)))
    flat = P.Volume(dims, tuple(grid.origin), grid.voxel, grid.trunc, device=DEV, skip_bricks=False)
    flat.tsdf.copy_(dense.tsdf)
    flat.rgb.copy_(dense.rgb)
    rng = np.random.Generator(np.random.PCG64(5))
    for skip, ranged in ((True, True), (True, False), (False, True), (False, False)):
        vol_b = vol.block_min
        if not skip:
            vol.block_min = None
        outs = P.hash_raycast(vol, cams, z_near=z_near, range_scratch=ranged)
        vol.block_min = vol_b
        dref = P.raycast(dense if skip else flat, cams, z_near=z_near)
        torch.cuda.synchronize()
        for cam, (hd, hc), (dd, dc) in zip(cams, outs, dref):
            np.testing.assert_array_equal(h(hd), h(dd))
            np.testing.assert_array_equal(h(hc), h(dc))
            if not ranged:
                continue
            HW = cam["width"] * cam["height"]
            pix = None if n_sample is None else np.sort(rng.choice(HW, n_sample, replace=False)).astype(np.int32)
            rd, rc, rk = O.raycast(grid, t32, c32, cam, z_near=z_near, pix=pix)
            gd = h(hd).reshape(-1) if pix is None else h(hd).reshape(-1)[pix]
            gc = h(hc).reshape(3, -1) if pix is None else h(hc).reshape(3, -1)[:, pix]
            assert ((gd > 0) == (rk >= 0)).mean() >= 0.999
            both = (gd > 0) & (rk >= 0)
            assert (rk >= 0).sum() > 1000 and both.sum() >= 0.999 * (rk >= 0).sum()
            assert np.abs(gd[both] - rd[both]).max() <= 1e-4 * rd[both].max()
            assert np.abs(gc[:, both] - rc[:, both]).max() <= 1e-3


def test_hash_small_scene(P, O):
    say("hash: 64^3 scene, one 160x120 frame")
    w = synth.workload_small(M=10)
    sc, cam = w["scene"], w["cam"].as_dict()
    vol = P.HashVolume(sc.dims, sc.origin, sc.voxel, sc.trunc, capacity=1024)
    P.hash_fuse(vol, cam, t(w["depth"]), t(w["rgb"]))
    torch.cuda.synchronize()
    st = vol.state()
    assert st["status"] == 0 and st["allocated"] > 50 and st["visible"] == st["allocated"]
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    mask = O.alloc_blocks(grid, cam, w["depth"])
    ref = O.fuse(grid, O.new_volume(grid), cam, w["depth"], w["rgb"], block_mask=mask)
    _check_volume(O, vol, grid, ref, mask, 2e-5)
    t32, c32 = ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32)
    _raycast_checks(P, O, vol, grid, sc.dims, [cam], t32, c32)
    say(f"  blocks {st['allocated']}, pool {st['allocated'] * 512 * 24 / 1e6:.1f} MB against "
        f"{np.prod(sc.dims) * 24 / 1e6:.1f} MB dense")


def test_hash_room_frames(P, O):
    say("hash: 256^3 room, three 1280x720 frames")
    scene, fr = synth.workload_room_frames(n=256, frames=[0, 10, 20])
    vol = P.HashVolume(scene.dims, scene.origin, scene.voxel, scene.trunc, capacity=60_000)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    mask = None
    ref = O.new_volume(grid)
    for cam, d, c in fr:
        camd = cam.as_dict()
        P.hash_fuse(vol, camd, t(d), t(c))
        mask = O.alloc_blocks(grid, camd, d, mask=mask)
        O.fuse(grid, ref, camd, d, c, block_mask=mask)
        torch.cuda.synchronize()
        st = vol.state()
        assert st["status"] == 0
        assert _mask_set(mask) == {tuple(b) for b in _blocks(vol).T.tolist()}
    _check_volume(O, vol, grid, ref, mask, 1e-4)
    say(f"  blocks {st['allocated']} ({st['allocated'] * 512 * 24 / 1e6:.0f} MB of pool against "
        f"{np.prod(scene.dims) * 24 / 1e6:.0f} MB dense), visible in the last frame {st['visible']}")
    t32, c32 = ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32)
    _raycast_checks(P, O, vol, grid, scene.dims, [cam.as_dict() for cam, _, _ in fr], t32, c32, n_sample=3000)


def test_hash_refusion_and_overflow(P, O):
    say("hash: the same frame twice; a pool too small")
    w = synth.workload_small(M=10)
    sc, cam = w["scene"], w["cam"].as_dict()
    vol = P.HashVolume(sc.dims, sc.origin, sc.voxel, sc.trunc, capacity=1024)
    for _ in range(2):
        P.hash_fuse(vol, cam, t(w["depth"]), t(w["rgb"]))
    torch.cuda.synchronize()
    st = vol.state()
    assert st["allocated"] == st["allocated_before"] and st["status"] == 0
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    mask = O.alloc_blocks(grid, cam, w["depth"])
    ref = O.new_volume(grid)
    for _ in range(2):
        O.fuse(grid, ref, cam, w["depth"], w["rgb"], block_mask=mask)
    _check_volume(O, vol, grid, ref, mask, 2e-5)
    # overflow: a pool of 16 blocks keeps 16, flags the rest; the stored blocks stay valid
    small = P.HashVolume(sc.dims, sc.origin, sc.voxel, sc.trunc, capacity=16)
    P.hash_fuse(small, cam, t(w["depth"]), t(w["rgb"]))
    torch.cuda.synchronize()
    st = small.state()
    assert st["status"] & 1 and st["allocated"] > 16
    bc = _blocks(small)
    assert bc.shape[1] == 16 and {tuple(b) for b in bc.T.tolist()} <= _mask_set(mask)
    P.hash_raycast(small, [cam])  # reads the blocks without room as unallocated
    small.reset()
    torch.cuda.synchronize()
    assert small.state() == {"allocated": 0, "allocated_before": 0, "visible": 0, "status": 0}
    assert (small.keys.cpu().numpy().view(np.uint64) == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
