"""Forward-only render server over a resident triangle soup: continuous
batching of camera requests into HIP-graph replays of the batched renderer,
and the one-view-per-launch baseline it is compared with."""
