"""Oracle of the densification step (Sec. 3.2, "Densification"; Supp.,
"Densification") -- TEST INFRASTRUCTURE ONLY: only the test suite and the
benchmark's CPU-baseline leg may import this module.  Plain numpy in float64
(float32 where the inputs are float32 and the result is exact); it shares no
code with the HIP path.

What it computes:
  - the sampling distribution of a densification step, built from the
    triangles' own parameters: weight o_i (opacity) or 1/sigma_i (the
    inverse sharpness, which favours solid triangles), the two used in
    alternate steps;
  - Bernoulli sampling: triangle i is selected independently with
    probability p_i = min(1, k w_i / sum_j w_j), so k triangles are
    selected on average (exactly sum_i p_i);
  - midpoint subdivision of every selected triangle into four, joining the
    midpoints of its edges: the four children cover exactly the parent's
    region and each has a quarter of its area.  Children inherit the
    parent's opacity, sigma and SH coefficients.

Layout of the subdivided soup (a reading; the paper fixes none): the centre
child (m01, m12, m20) replaces the parent at its index; the corner children
(v0, m01, m20), (m01, v1, m12), (m20, m12, v2) follow the N input triangles
at N + 3 r, N + 3 r + 1, N + 3 r + 2, r the number of selected triangles
before it.  Uniform random numbers are inputs, so both implementations
draw the same sample.
"""
from __future__ import annotations

import numpy as np

OPACITY = 0
INV_SIGMA = 1


def weights(o, sigma, mode: int) -> np.ndarray:
    """w_i = o_i (mode 0) or 1/sigma_i (mode 1), float64."""
    if mode == OPACITY:
        return np.asarray(o, np.float64).copy()
    return 1.0 / np.asarray(sigma, np.float64)


def probabilities(o, sigma, mode: int, k: float) -> np.ndarray:
    """p_i = min(1, k w_i / sum_j w_j) (zeros when the sum is not positive)."""
    w = weights(o, sigma, mode)
    tot = float(np.sum(w))
    if not tot > 0.0:
        return np.zeros_like(w)
    return np.minimum(1.0, k * w / tot)


def select(o, sigma, mode: int, k: float, u) -> np.ndarray:
    """Bernoulli sampling: selected where u_i < p_i (u uniform in [0, 1))."""
    return np.asarray(u, np.float64) < probabilities(o, sigma, mode, k)


def midpoint_children(tri) -> np.ndarray:
    """The four children of one triangle [3,3] (or a batch [n,3,3]):
    [centre, corner at v0, corner at v1, corner at v2], each [3,3].
    Midpoints are computed in the input precision: (a + b) / 2 is exact up
    to one rounding."""
    t = np.asarray(tri)
    v0, v1, v2 = t[..., 0, :], t[..., 1, :], t[..., 2, :]
    half = t.dtype.type(0.5)
    m01, m12, m20 = (v0 + v1) * half, (v1 + v2) * half, (v2 + v0) * half
    return np.stack([np.stack([m01, m12, m20], -2),
                     np.stack([v0, m01, m20], -2),
                     np.stack([m01, v1, m12], -2),
                     np.stack([m20, m12, v2], -2)], -3)


def subdivide(v, o, sigma, sh, sel):
    """The soup after midpoint subdivision of the selected triangles, in the
    layout described above.  Returns (v, o, sigma, sh) with N + 3 n_sel
    triangles."""
    v = np.asarray(v)
    sel = np.asarray(sel, bool)
    idx = np.nonzero(sel)[0]
    N, n = v.shape[0], idx.size
    out_v = np.concatenate([v, np.zeros((3 * n, 3, 3), v.dtype)])
    out_o = np.concatenate([o, np.zeros(3 * n, np.asarray(o).dtype)])
    out_s = np.concatenate([sigma, np.zeros(3 * n, np.asarray(sigma).dtype)])
    out_sh = np.concatenate([sh, np.zeros((3 * n,) + np.asarray(sh).shape[1:], np.asarray(sh).dtype)])
    ch = midpoint_children(v[idx])            # [n, 4, 3, 3]
    out_v[idx] = ch[:, 0]
    for c in range(3):                         # corner c of the r-th selected: N + 3 r + c
        j = N + 3 * np.arange(n) + c
        out_v[j] = ch[:, 1 + c]
        out_o[j], out_s[j], out_sh[j] = np.asarray(o)[idx], np.asarray(sigma)[idx], np.asarray(sh)[idx]
    return out_v, out_o, out_s, out_sh
