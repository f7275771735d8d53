"""GPU parity of the differentiable wrapper: gradients that reach the leaf
tensors through `rasterize()` (the torch.autograd.Function with transmittance
recovered from the final T) against the FP64 oracle gradient (Sec. 3.3,
end-to-end optimisation of every triangle parameter).

The loss is L = sum dC.rgb + dA.alpha + dD.depth with seeded N(0,1) upstream
arrays, zeroed on pixels the oracle flags (a decision within a rounding band
of its threshold).  Bars: per element |delta| <= 1e-3 |ref| + 1e-6 max|ref of
the group| and relative L2 <= 1e-3 for v, o, sigma and sh."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_19175_amd import synth
from paper_2505_19175_amd.autograd import rasterize

import gpu_util as G

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _leaves(scene):
    return tuple(torch.tensor(a, device=DEV, dtype=torch.float32, requires_grad=True)
                 for a in (scene.v, scene.o, scene.sigma, scene.sh))


def _grads(leaves):
    return {k: t.grad.detach().cpu().numpy().astype(np.float64)
            for k, t in zip(("v", "o", "sigma", "sh"), leaves)}


def _upstream(wl, cam, ref, alpha, depth):
    dC, dA, dD = synth.upstream(wl.upstream_seed, cam.width, cam.height, alpha, depth)
    keep = ref["flag"] == 0
    dC = dC * keep[None]
    dA = None if dA is None else dA * keep
    dD = None if dD is None else dD * keep
    return dC, dA, dD


def _run(wl, use_rgb=True, use_alpha=True, use_depth=True):
    scene, cam, cfg = wl.scene, wl.cameras[0], wl.config
    ref = O.render(scene, cam, cfg)
    dC, dA, dD = _upstream(wl, cam, ref, use_alpha, use_depth)
    leaves = _leaves(scene)
    rgb, alpha, depth = rasterize(*leaves, cam, cfg)
    G.assert_forward({"rgb": rgb.detach().cpu().numpy().astype(np.float64),
                      "alpha": alpha.detach().cpu().numpy().astype(np.float64),
                      "depth": depth.detach().cpu().numpy().astype(np.float64),
                      "T_final": 1.0 - alpha.detach().cpu().numpy().astype(np.float64)}, ref)
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=DEV)
    terms = []
    if use_rgb:
        terms.append((rgb * t(dC)).sum())
    if use_alpha:
        terms.append((alpha * t(dA)).sum())
    if use_depth:
        terms.append((depth * t(dD)).sum())
    sum(terms).backward()
    torch.cuda.synchronize()
    r = O.backward(scene, cam, cfg, dC if use_rgb else np.zeros_like(dC), dA, dD)
    return _grads(leaves), r


def test_autograd_small_all_outputs():
    """1k triangles, 128x128, SH degree 0: loss over rgb, alpha and depth."""
    wl = synth.workload_small()
    g, r = _run(wl)
    print("autograd small", G.assert_grads(g, r))


@pytest.mark.parametrize("sigma", [0.25, 1.0, 4.0])
def test_autograd_grad_workload(sigma):
    """20k triangles, 256x256, SH degree 1, sigma swept: every parameter
    group through the autograd.Function against the oracle."""
    wl = synth.workload_grad(sigma)
    g, r = _run(wl)
    print("autograd grad workload", sigma, G.assert_grads(g, r))


@pytest.mark.parametrize("outputs", [(True, False, False), (True, True, False),
                                     (True, False, True), (False, True, False),
                                     (False, False, True)])
def test_autograd_unused_outputs(outputs):
    """Outputs left out of the loss reach the backward as None (alpha,
    depth) or are replaced by zeros (rgb); the gradient is the oracle's for
    the terms that are present."""
    wl = synth.workload_grad(1.0)
    g, r = _run(wl, *outputs)
    print("autograd unused outputs", outputs, G.assert_grads(g, r))


def test_autograd_retained_graph_twice():
    """A retained graph runs the backward twice; the second pass adds the
    same gradient again (the per-triangle accumulators are clean again after
    each backward), up to the order of the FP32 atomic sums."""
    wl = synth.workload_small()
    scene, cam, cfg = wl.scene, wl.cameras[0], wl.config
    leaves = _leaves(scene)
    rgb, alpha, depth = rasterize(*leaves, cam, cfg)
    dC, _, _ = synth.upstream(wl.upstream_seed, cam.width, cam.height)
    loss = (rgb * torch.tensor(dC, device=DEV)).sum() + alpha.sum()
    loss.backward(retain_graph=True)
    first = _grads(leaves)
    loss.backward()
    second = _grads(leaves)
    G.assert_grads({k: second[k] - first[k] for k in first}, first)


def test_autograd_no_double_backward():
    wl = synth.workload_small(200)
    scene, cam, cfg = wl.scene, wl.cameras[0], wl.config
    leaves = _leaves(scene)
    rgb, _, _ = rasterize(*leaves, cam, cfg)
    (gv,) = torch.autograd.grad(rgb.sum(), leaves[0], create_graph=True)
    with pytest.raises(RuntimeError):
        gv.sum().backward()


def test_autograd_rejects_bad_inputs():
    wl = synth.workload_small(100)
    scene, cam, cfg = wl.scene, wl.cameras[0], wl.config
    v, o, s, sh = _leaves(scene)
    with pytest.raises(ValueError):        # SH rows of the wrong degree
        rasterize(v, o, s, torch.zeros((scene.n, 4, 3), device=DEV), cam, cfg)
    with pytest.raises(ValueError):        # opacity of the wrong length
        rasterize(v, o[:-1], s, sh, cam, cfg)
    with pytest.raises(ValueError):        # a host tensor
        rasterize(v, o.detach().cpu(), s, sh, cam, cfg)
    with pytest.raises(ValueError):        # vertices not [N,3,3]
        rasterize(v.reshape(-1, 9), o, s, sh, cam, cfg)
