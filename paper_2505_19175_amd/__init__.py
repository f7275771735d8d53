"""MI355X-native (gfx950) differentiable triangle-splatting rasterizer.

The compute path is the C-ABI library `libts.so` (hand-written HIP kernels
for projection + SH colour, tile binning with a device radix sort, forward
and backward tile compositing).  Importing the package does not load it;
`paper_2505_19175_amd.binding` does, and raises if it is missing.
"""
__all__ = ["synth"]
