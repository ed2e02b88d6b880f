"""The reference implementation gives bitwise the same results on one thread and on
several (fusion, raycast, render and backward run their independent pixels or lattice
points on OpenMP threads; the backward adds the pixels' adjoints in pixel order)."""
import numpy as np

from tests.tiny_cases import tiny_case


def test_results_do_not_depend_on_the_thread_count(oracle, small_workload):
    O = oracle
    n0 = O.set_threads()
    w = small_workload
    sc, cam = w["scene"], w["cam"]
    case = tiny_case(3, M=80, W=53, H=37, log_scale=-2.4)
    rng = np.random.default_rng(1)
    gC, gD = rng.normal(size=(3, 53 * 37)), rng.normal(size=53 * 37)
    runs = []
    try:
        for n in (1, max(2, n0)):
            assert O.set_threads(n) == n
            grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
            vol = O.fuse(grid, O.new_volume(grid), cam.as_dict(), w["depth"], w["rgb"])
            rd, rc, rk = O.raycast(grid, vol["tsdf"].astype(np.float32), vol["rgb"].astype(np.float32), cam.as_dict())
            out = {"tsdf": vol["tsdf"], "rd": rd, "rc": rc, "rk": rk}
            for mode in (0, 1):
                cfg = O.RenderCfg(mode=mode, eps_cull=0.03)
                r = O.render(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
                g = O.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
                out.update({f"{k}{mode}": v for k, v in r.items()})
                out.update({f"g{k}{mode}": v for k, v in g.items()})
            runs.append(out)
    finally:
        O.set_threads(n0)
    for k in runs[0]:
        np.testing.assert_array_equal(runs[0][k], runs[1][k], err_msg=k)
