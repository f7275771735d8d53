"""Oracle of one synthetic training step (Sec. 3.3, "Optimization"; Supp.
hyperparameters) -- TEST INFRASTRUCTURE ONLY: only the test suite and the
benchmark's CPU-baseline leg may import this module.  Plain numpy/scipy in
float64; it shares no code with the HIP path.

What it computes, with the choices the paper leaves to the works it cites:
  - the photometric loss (1 - lambda) L1 + lambda (1 - SSIM) between the
    rendered image C [3,H,W] and a target: L1 the mean absolute difference
    over pixels and channels; SSIM per channel with an 11x11 Gaussian window
    of standard deviation 1.5 (sum 1), constants C1 = 0.01^2, C2 = 0.03^2,
    the window zero-padded at the image border, averaged over pixels and
    channels; lambda = 0.2 (the 3D Gaussian Splatting setting it cites);
  - the opacity loss L_o = mean_i o_i and the size loss
    L_s = mean_i 2 / |(v1 - v0) x (v2 - v0)| (the inverse area of each
    triangle), weighted by beta_1 and beta_4 from the hyperparameter table
    (lambda_opacity = 0.0055, lambda_size = 1e-8 outdoor);
  - the gradient of all of it: of the image loss w.r.t. C by the chain rule
    through the five local statistics of SSIM (pinned by finite
    differences), of L_o and L_s w.r.t. o and the vertices;
  - Adam (beta = (0.9, 0.999), eps = 1e-15, bias-corrected) on the raw
    parameters: vertices; opacity through o = sigmoid(a); sigma through
    sigma = exp(b); SH coefficients, the degree-0 ones at feature_lr and the
    rest at feature_lr / 20; learning rates from the hyperparameter table.
The distortion and normal losses (which need rendered depth distortion and
normal maps) are not part of this step.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import correlate2d

LAMBDA_DSSIM = 0.2
C1 = 0.01 ** 2
C2 = 0.03 ** 2
BETA_OPACITY = 0.0055
BETA_SIZE = 1e-8
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-15
LR = {"v": 0.0018, "o": 0.014, "sigma": 0.0008, "sh_dc": 0.0025, "sh_rest": 0.0025 / 20.0}


def gaussian_window(size: int = 11, std: float = 1.5) -> np.ndarray:
    x = np.arange(size, dtype=np.float64) - (size // 2)
    g = np.exp(-x * x / (2.0 * std * std))
    g /= g.sum()
    return np.outer(g, g)


def _blur(img: np.ndarray) -> np.ndarray:
    """Local mean under the Gaussian window, zero outside the image."""
    return correlate2d(img, gaussian_window(), mode="same", boundary="fill", fillvalue=0.0)


def _stats(x, y):
    mx, my = _blur(x), _blur(y)
    exx, eyy, exy = _blur(x * x), _blur(y * y), _blur(x * y)
    return mx, my, exx - mx * mx, eyy - my * my, exy - mx * my


def ssim_map(x, y) -> np.ndarray:
    """SSIM of each pixel of each channel, images [3,H,W]."""
    out = np.empty(np.shape(x))
    for c in range(np.shape(x)[0]):
        mx, my, vx, vy, cxy = _stats(np.asarray(x[c], np.float64), np.asarray(y[c], np.float64))
        out[c] = ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    return out


def image_loss(C, target, lam: float = LAMBDA_DSSIM) -> float:
    C = np.asarray(C, np.float64)
    T = np.asarray(target, np.float64)
    return float((1 - lam) * np.mean(np.abs(C - T)) + lam * (1.0 - np.mean(ssim_map(C, T))))


def image_loss_grad(C, target, lam: float = LAMBDA_DSSIM) -> np.ndarray:
    """dL/dC.  SSIM at q depends on x = C through mu_x(q), E[x^2](q) and
    E[xy](q), each a window sum over pixels p, so dS(q)/dx(p) =
    w(q - p) (dS/dmu_x + 2 x(p) dS/dE[x^2] + y(p) dS/dE[xy]) at q; summing
    over q is again a zero-padded blur (the window is symmetric).  The L1
    term uses sign(0) = 0."""
    C = np.asarray(C, np.float64)
    T = np.asarray(target, np.float64)
    n = C.size
    g = (1 - lam) * np.sign(C - T) / n
    for c in range(C.shape[0]):
        x, y = C[c], T[c]
        mx, my, vx, vy, cxy = _stats(x, y)
        A = 2 * mx * my + C1
        Bn = 2 * cxy + C2
        D1 = mx * mx + my * my + C1
        D2 = vx + vy + C2
        S = A * Bn / (D1 * D2)
        # partial derivatives of S w.r.t. (mu_x, var_x, cov_xy)
        dS_dmx = 2 * my * Bn / (D1 * D2) - S * 2 * mx / D1
        dS_dvx = -S / D2
        dS_dcxy = 2 * A / (D1 * D2)
        # to the raw moments: var_x = E[x^2] - mu_x^2, cov = E[xy] - mu_x mu_y
        d_mx = dS_dmx - 2 * mx * dS_dvx - my * dS_dcxy
        d_exx = dS_dvx
        d_exy = dS_dcxy
        up = -lam / n
        g[c] += up * (_blur(d_mx) + 2 * x * _blur(d_exx) + y * _blur(d_exy))
    return g


def size_loss(v) -> float:
    v = np.asarray(v, np.float64)
    cr = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    return float(np.mean(2.0 / np.linalg.norm(cr, axis=1)))


def size_loss_grad(v) -> np.ndarray:
    """d/dv of mean_i 2 / |c_i|, c = (v1 - v0) x (v2 - v0):
    d(2/|c|) = -2 c . dc / |c|^3, dc/dv1 = [(v2 - v0)]_x^T-style terms."""
    v = np.asarray(v, np.float64)
    N = v.shape[0]
    e1, e2 = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]
    cr = np.cross(e1, e2)
    nrm = np.linalg.norm(cr, axis=1)
    gc = (-2.0 / nrm ** 3)[:, None] * cr / N         # dL/dc
    g1 = np.cross(e2, gc)                            # c = e1 x e2: dL/de1 = e2 x gc
    g2 = np.cross(gc, e1)                            #              dL/de2 = gc x e1
    out = np.zeros_like(v)
    out[:, 1] = g1
    out[:, 2] = g2
    out[:, 0] = -g1 - g2
    return out


def adam(p, g, m, s, lr: float, t: int, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One bias-corrected Adam update (step t >= 1); returns (p, m, s)."""
    m = b1 * m + (1 - b1) * g
    s = b2 * s + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    sh = s / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(sh) + eps), m, s


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-np.asarray(a, np.float64)))


def optimizer_step(raw: dict, grads: dict, state: dict, t: int, lr: dict = LR,
                   beta_o: float = BETA_OPACITY, beta_s: float = BETA_SIZE):
    """raw: {"v" [N,3,3], "a" [N] opacity logit, "b" [N] log sigma, "sh" [N,K,3]};
    grads: the renderer's {"v", "o", "sigma", "sh"} w.r.t. o and sigma;
    state: Adam moments {name: (m, s)}.  Adds the regularizer gradients,
    chains through the activations and returns (raw, state) after one step."""
    v = np.asarray(raw["v"], np.float64)
    o = sigmoid(raw["a"])
    sig = np.exp(np.asarray(raw["b"], np.float64))
    N = v.shape[0]
    gv = np.asarray(grads["v"], np.float64).reshape(N, 3, 3) + beta_s * size_loss_grad(v)
    go = np.asarray(grads["o"], np.float64) + beta_o / N
    ga = go * o * (1 - o)
    gb = np.asarray(grads["sigma"], np.float64) * sig
    gsh = np.asarray(grads["sh"], np.float64).reshape(np.shape(raw["sh"]))
    out, new_state = {}, {}
    for name, p, g, rate in (("v", v, gv, lr["v"]), ("a", raw["a"], ga, lr["o"]),
                             ("b", raw["b"], gb, lr["sigma"])):
        m, s = state[name]
        out[name], m, s = adam(np.asarray(p, np.float64), g, m, s, rate, t)
        new_state[name] = (m, s)
    sh = np.asarray(raw["sh"], np.float64)
    m, s = state["sh"]
    rate = np.full(sh.shape, lr["sh_rest"])
    rate[:, 0, :] = lr["sh_dc"]
    out["sh"], m, s = adam(sh, gsh, m, s, rate, t)
    new_state["sh"] = (m, s)
    return out, new_state
