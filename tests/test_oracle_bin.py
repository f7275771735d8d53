"""Pin of the oracle's tile binning (Supp. 'Tile assignment' and 'Depth
sorting'): the vectorised emission + lexsort equals a brute-force loop over
triangles and tiles followed by Python's sort of (tile, depth key, index)."""
import struct

import numpy as np

from oracle import oracle as O
from paper_2505_19175_amd.synth import Config

from helpers import random_soup


def _brute(st, W, H):
    tx_n = (W + 15) // 16
    inst = []
    for i in range(len(st["ntiles"])):
        if st["ntiles"][i] == 0:
            continue
        px0, px1, py0, py1 = st["rect"][i]
        kb = struct.unpack("<I", struct.pack("<f", float(st["key"][i])))[0]
        for ty in range(py0 // 16, py1 // 16 + 1):
            for tx in range(px0 // 16, px1 // 16 + 1):
                inst.append((ty * tx_n + tx, kb, i))
    inst.sort()
    return inst


def test_binning_matches_brute_force():
    sc, cam = random_soup(31, 400, W=100, H=70, size=2.5, deg=0)
    cfg = Config(sh_degree=0)
    b = O.bin_instances(sc, cam, cfg)
    inst = _brute(b["setup"], 100, 70)
    assert b["count"] == len(inst) > 400
    keys = np.array([(t << 32) | k for t, k, _ in inst], np.uint64)
    vals = np.array([i for _, _, i in inst], np.uint32)
    np.testing.assert_array_equal(b["keys"], keys)
    np.testing.assert_array_equal(b["vals"], vals)
    # ranges: [start, end) of each tile's run in the sorted list
    tiles = np.array([t for t, _, _ in inst])
    for t in range(b["n_tiles"]):
        pos = np.nonzero(tiles == t)[0]
        if len(pos) == 0:
            assert tuple(b["ranges"][t]) == (0, 0)
        else:
            assert tuple(b["ranges"][t]) == (pos[0], pos[-1] + 1)


def test_binned_instances_cover_contributing_pixels():
    """Every pixel a triangle contributes to (in the brute-force render) lies
    in a tile that lists the triangle."""
    sc, cam = random_soup(32, 60, W=64, H=48, size=1.5, deg=0)
    cfg = Config(sh_degree=0)
    b = O.bin_instances(sc, cam, cfg)
    st = b["setup"]
    tx_n = 4
    listed = {}
    for t in range(b["n_tiles"]):
        s, e = b["ranges"][t]
        listed[t] = set(b["vals"][s:e].tolist())
    amin = float(np.float32(cfg.alpha_min))
    for i in range(sc.n):
        if not st["vis"][i]:
            continue
        for y in range(48):
            for x in range(64):
                u, I = O.window(st["q"][i], (x + 0.5, y + 0.5), float(sc.sigma[i]))
                if float(sc.o[i]) * I >= amin * (1 + 1e-9):
                    assert i in listed[(y // 16) * tx_n + x // 16]
