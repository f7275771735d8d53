"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP path: it loads
`libts_oracle.so`, built from `ts_oracle.c` in this directory with gcc, and
performs the tile binning of the supplementary "Tile assignment" and
"Depth sorting" paragraphs in plain numpy.

Inputs are the float32 arrays of `paper_2505_19175_amd.synth` (Scene,
Camera, Config); the oracle reads them exactly (float32 -> float64) and
computes in double precision.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ts_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libts_oracle.so")
_lib = None

TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _configure(L):
    P = ctypes.c_void_p
    L.oracle_setup.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                               ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P]
    L.oracle_window.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, P, P]
    L.oracle_sh.argtypes = [ctypes.c_int, P, P, P]
    L.oracle_render.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P, P, P, P]
    L.oracle_backward.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                  ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P, P, P, P]
    L.oracle_prune_stats.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                     ctypes.c_int, P, ctypes.c_int64, P, P, P]
    L.oracle_render_flip.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, ctypes.c_int,
                                     ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P, P, P]
    L.oracle_threads.argtypes = []
    for f in (L.oracle_setup, L.oracle_window, L.oracle_sh, L.oracle_render,
              L.oracle_render_flip, L.oracle_backward, L.oracle_prune_stats, L.oracle_threads):
        f.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


class use_library:
    """Context manager: route every call through another build of the
    oracle (used to check that the pins catch planted mistakes)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _configure(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def threads() -> int:
    return int(lib().oracle_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _cam16(cam) -> np.ndarray:
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(9)
    t = np.asarray(cam.t, np.float32).astype(np.float64).reshape(3)
    rest = np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32).astype(np.float64)
    return np.ascontiguousarray(np.concatenate([R, t, rest]))


def _cfg9(cfg) -> np.ndarray:
    vals = [cfg.alpha_min, cfg.alpha_max, cfg.T_min, cfg.z_near, cfg.r_min] + list(cfg.bg)
    out = np.array(vals, np.float32).astype(np.float64)
    return np.ascontiguousarray(np.append(out, float(getattr(cfg, "window", 0))))


def _scene_arrays(scene):
    v = _d(scene.v).reshape(-1)
    o = _d(scene.o)
    s = _d(scene.sigma)
    sh = _d(scene.sh).reshape(-1)
    return v, o, s, sh


def _deg(scene, cfg) -> int:
    deg = int(cfg.sh_degree)
    K = (deg + 1) ** 2
    if scene.sh.shape[1] != K:
        raise ValueError(f"scene has {scene.sh.shape[1]} SH coefficients, config degree {deg}")
    return deg


# ---------------------------------------------------------------------------

def setup(scene, cam, cfg) -> dict:
    """Per-triangle quantities: vis, q[N,3,2], r, s[N,2], phis, zc, key (f32),
    rgb[N,3], rect[N,4] (px0,px1,py0,py1; empty = (0,-1,0,-1)), ntiles."""
    N = scene.n
    v, o, s, sh = _scene_arrays(scene)
    out = dict(vis=np.zeros(N, np.int32), q=np.zeros((N, 3, 2)), r=np.zeros(N),
               s=np.zeros((N, 2)), phis=np.zeros(N), zc=np.zeros(N),
               key=np.zeros(N, np.float32), rgb=np.zeros((N, 3)),
               rect=np.zeros((N, 4), np.int32), ntiles=np.zeros(N, np.int32))
    rc = lib().oracle_setup(N, _p(v), _p(o), _p(s), _p(sh), _deg(scene, cfg), _p(_cam16(cam)),
                            cam.width, cam.height, _p(_cfg9(cfg)), _p(out["vis"]), _p(out["q"]),
                            _p(out["r"]), _p(out["s"]), _p(out["phis"]), _p(out["zc"]),
                            _p(out["key"]), _p(out["rgb"]), _p(out["rect"]), _p(out["ntiles"]))
    assert rc == 0
    return out


def window(q, p, sigma: float, window: int = 0):
    """(u, I) at point p for one 2D triangle q[3,2]: window 0 is Eq. 1
    (u = phi(p)/phi(s)), 1 the sigmoid of Eq. 2 (u = phi(p)), 2 Eq. 1 with
    the LogSumExp SDF (u = phi_lse(p)/phi_lse(s))."""
    q6 = _d(q).reshape(6)
    u = ctypes.c_double()
    I = ctypes.c_double()
    lib().oracle_window(_p(q6), float(p[0]), float(p[1]), float(sigma), int(window),
                        ctypes.byref(u), ctypes.byref(I))
    return u.value, I.value


def sh_basis(deg: int, direction, grad: bool = False):
    K = (deg + 1) ** 2
    d = _d(direction).reshape(3)
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    rc = lib().oracle_sh(deg, _p(d), _p(Y), _p(dY))
    assert rc == 0
    return (Y, dY) if grad else Y


def render(scene, cam, cfg, pix: Optional[np.ndarray] = None) -> dict:
    """Forward render.  pix = linear pixel indices (y*W+x) or None (full
    frame).  Full frame outputs are shaped [3,H,W] / [H,W]; sampled outputs
    [3,npix] / [npix]."""
    N = scene.n
    v, o, s, sh = _scene_arrays(scene)
    pixa = None if pix is None else np.ascontiguousarray(pix, np.int64)
    npix = cam.width * cam.height if pixa is None else pixa.size
    rgb = np.zeros(3 * npix)
    alpha = np.zeros(npix)
    depth = np.zeros(npix)
    Tf = np.zeros(npix)
    nfrag = np.zeros(npix, np.int32)
    flag = np.zeros(npix, np.int32)
    hsh = np.zeros(npix, np.uint64)
    rc = lib().oracle_render(N, _p(v), _p(o), _p(s), _p(sh), _deg(scene, cfg), _p(_cam16(cam)),
                             cam.width, cam.height, _p(_cfg9(cfg)), npix, _p(pixa), _p(rgb),
                             _p(alpha), _p(depth), _p(Tf), _p(nfrag), _p(flag), _p(hsh))
    assert rc == 0
    out = dict(rgb=rgb.reshape(3, npix), alpha=alpha, depth=depth, T_final=Tf,
               nfrag=nfrag, flag=flag, hash=hsh)
    if pixa is None:
        H, W = cam.height, cam.width
        out = {k: (a.reshape(3, H, W) if k == "rgb" else a.reshape(H, W)) for k, a in out.items()}
    return out


def render_flip(scene, cam, cfg, pix: np.ndarray, flips: np.ndarray) -> dict:
    """Forward render of the listed pixels, each with a mask of its
    near-threshold decisions (alpha against alpha_min, T(1-alpha) against
    T_min, numbered in walk order) taken the other way.  Both outcomes of
    such a decision are correct renders (a rounding difference picks one);
    flips = 0 gives render()'s result.  Returns rgb [3,npix], alpha, depth,
    T_final and ndec (the number of such decisions met)."""
    N = scene.n
    v, o, s, sh = _scene_arrays(scene)
    pixa = np.ascontiguousarray(pix, np.int64)
    fl = np.ascontiguousarray(flips, np.uint32)
    assert fl.shape == pixa.shape
    npix = pixa.size
    rgb = np.zeros(3 * npix)
    alpha = np.zeros(npix)
    depth = np.zeros(npix)
    Tf = np.zeros(npix)
    ndec = np.zeros(npix, np.int32)
    rc = lib().oracle_render_flip(N, _p(v), _p(o), _p(s), _p(sh), _deg(scene, cfg),
                                  _p(_cam16(cam)), cam.width, cam.height, _p(_cfg9(cfg)), npix,
                                  _p(pixa), _p(fl), _p(rgb), _p(alpha), _p(depth), _p(Tf),
                                  _p(ndec))
    assert rc == 0
    return dict(rgb=rgb.reshape(3, npix), alpha=alpha, depth=depth, T_final=Tf, ndec=ndec)


def prune_stats(scene, cam, cfg, pix: Optional[np.ndarray] = None) -> dict:
    """Pruning statistics of one view (Sec. 3.2, "Pruning"): per triangle the
    largest T*o at its composited fragments and the number of pixels where it
    is composited, over the given pixels (default: all)."""
    N = scene.n
    v, o, s, sh = _scene_arrays(scene)
    pixa = None if pix is None else np.ascontiguousarray(pix, np.int64)
    npix = cam.width * cam.height if pixa is None else pixa.size
    maxw = np.zeros(max(N, 1))
    npx = np.zeros(max(N, 1), np.int32)
    rc = lib().oracle_prune_stats(N, _p(v), _p(o), _p(s), _p(sh), _deg(scene, cfg),
                                  _p(_cam16(cam)), cam.width, cam.height, _p(_cfg9(cfg)), npix,
                                  _p(pixa), _p(maxw), _p(npx))
    assert rc == 0
    return dict(max_weight=maxw[:N], pixels=npx[:N])


def backward(scene, cam, cfg, dC, dA=None, dD=None, pix: Optional[np.ndarray] = None) -> dict:
    """Analytic FP64 gradient of L = sum dC.rgb + dA.alpha + dD.depth over the
    given pixels (upstream arrays shaped like render()'s outputs)."""
    N = scene.n
    K = scene.sh.shape[1]
    v, o, s, sh = _scene_arrays(scene)
    pixa = None if pix is None else np.ascontiguousarray(pix, np.int64)
    npix = cam.width * cam.height if pixa is None else pixa.size
    dCf = _d(dC).reshape(3 * npix)
    dAf = None if dA is None else _d(dA).reshape(npix)
    dDf = None if dD is None else _d(dD).reshape(npix)
    gv = np.zeros(N * 9)
    go = np.zeros(N)
    gs = np.zeros(N)
    gsh = np.zeros(N * K * 3)
    rc = lib().oracle_backward(N, _p(v), _p(o), _p(s), _p(sh), _deg(scene, cfg), _p(_cam16(cam)),
                               cam.width, cam.height, _p(_cfg9(cfg)), npix, _p(pixa), _p(dCf),
                               _p(dAf), _p(dDf), _p(gv), _p(go), _p(gs), _p(gsh))
    assert rc == 0
    return dict(v=gv.reshape(N, 3, 3), o=go, sigma=gs, sh=gsh.reshape(N, K, 3))


def bin_instances(scene, cam, cfg) -> dict:
    """Tile binning (Supp., "Tile assignment" and "Depth sorting"): every
    triangle emits one instance per 16x16 tile of its tight pixel rectangle;
    instances are ordered by (tile, depth key, triangle index).  Returns
    keys (uint64: tile << 32 | float bits of the key), vals (uint32 triangle
    index), ranges [tiles,2] (start, end) and the per-triangle setup."""
    st = setup(scene, cam, cfg)
    W, H = cam.width, cam.height
    tx_n = (W + TILE - 1) // TILE
    ty_n = (H + TILE - 1) // TILE
    n_tiles = tx_n * ty_n
    idx = np.nonzero(st["ntiles"] > 0)[0]
    rect = st["rect"][idx]
    tx0, tx1 = rect[:, 0] // TILE, rect[:, 1] // TILE
    ty0, ty1 = rect[:, 2] // TILE, rect[:, 3] // TILE
    nx = tx1 - tx0 + 1
    cnt = nx * (ty1 - ty0 + 1)
    assert np.array_equal(cnt, st["ntiles"][idx])
    M = int(cnt.sum())
    tri = np.repeat(idx, cnt)
    # position of each instance inside its triangle's rectangle (row-major)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    j = np.arange(M) - start
    nxr = np.repeat(nx, cnt)
    tx = np.repeat(tx0, cnt) + j % nxr
    ty = np.repeat(ty0, cnt) + j // nxr
    tile = (ty * tx_n + tx).astype(np.uint64)
    kbits = st["key"].view(np.uint32)[tri].astype(np.uint64)
    order = np.lexsort((tri, kbits, tile))          # last key is primary
    keys = (tile[order] << np.uint64(32)) | kbits[order]
    vals = tri[order].astype(np.uint32)
    tiles_sorted = tile[order].astype(np.int64)
    ranges = np.zeros((n_tiles, 2), np.uint32)
    if M:
        first = np.searchsorted(tiles_sorted, np.arange(n_tiles), side="left")
        last = np.searchsorted(tiles_sorted, np.arange(n_tiles), side="right")
        ranges[:, 0] = first
        ranges[:, 1] = last
        empty = first == last
        ranges[empty] = 0
    return dict(keys=keys, vals=vals, ranges=ranges, count=M, n_tiles=n_tiles, setup=st)
