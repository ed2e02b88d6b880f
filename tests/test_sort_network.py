"""Host model of the per-tile register sorting network (k_tile_sort_small).

The kernel keeps element e = 64 r + lane in register r of lane `lane` and runs a
bitonic network whose merges start with a mirrored step (e <-> e ^ (k - 1)) and
continue with half-cleaners (e <-> e ^ j); every compare-exchange leaves the
smaller key at the lower index, and keys past the tile's length are +inf.  This
model applies the same exchanges to arrays of 64 lanes x R registers (lane
exchanges at distances below 64, register swaps above) and checks that the
result is the sorted input for every register count the kernel uses.
"""
import numpy as np
import pytest

INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def network(keys, R):
    P, n = 64 * R, len(keys)
    x = np.full((R, 64), INF, np.uint64)
    flat = x.reshape(-1)
    flat[:n] = keys  # element e = 64 r + lane
    lanes = np.arange(64)
    k = 2
    while k <= P:
        if k <= 64:  # mirrored step inside the lane dimension
            low = (lanes & (k >> 1)) == 0
            for r in range(R):
                o = x[r, lanes ^ (k - 1)]
                x[r] = np.where(low, np.minimum(x[r], o), np.maximum(x[r], o))
        else:  # mirrored step across registers: register r ^ jr of lane ^ 63
            jr = k // 64 - 1
            o = np.stack([x[r ^ jr, lanes ^ 63] for r in range(R)])
            for r in range(R):
                x[r] = np.minimum(x[r], o[r]) if ((64 * r) & (k >> 1)) == 0 else np.maximum(x[r], o[r])
        j = k >> 2
        while j > 0:
            if j >= 64:  # register swap
                jr = j // 64
                for r in range(R):
                    if r & jr == 0:
                        a, b = x[r].copy(), x[r | jr].copy()
                        x[r], x[r | jr] = np.minimum(a, b), np.maximum(a, b)
            else:  # lane exchange
                low = (lanes & j) == 0
                for r in range(R):
                    o = x[r, lanes ^ j]
                    x[r] = np.where(low, np.minimum(x[r], o), np.maximum(x[r], o))
            j >>= 1
        k <<= 1
    return x.reshape(-1)[:n]


@pytest.mark.parametrize("R", [1, 2, 4, 8])
def test_register_network_sorts(R):
    rng = np.random.default_rng(100 + R)
    for trial in range(40):
        n = int(rng.integers(2, 64 * R + 1)) if trial > 1 else (64 * R if trial == 0 else 2)
        keys = rng.integers(0, 1 << 62, n, dtype=np.uint64)
        if trial % 3 == 0:  # equal depths: ties broken by the low word
            keys = (keys & np.uint64(0xF00000000)) | rng.integers(0, 8, n).astype(np.uint64)
        np.testing.assert_array_equal(network(keys, R), np.sort(keys))
