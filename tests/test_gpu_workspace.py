"""Chunk workspaces kept per device between calls.

The fused estimator takes its chunk workspace from blocks the library keeps per device: a
later call gets a kept block back (the smallest idle one that fits) after waiting for the
block's last use on whatever stream, and a request larger than every idle block gives those
back and takes a new one.  Every sum has a fixed order, so the result of a call must not
depend on which block it gets, on the stream it runs on, or on the calls before it: bit for
bit.
"""

import numpy as np
import pytest
import torch

import paper_2408_16847_amd as z3
from synth import CONFIGS, make_positions, make_values
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def test_workspace_blocks_reused_across_streams_and_sizes():
    G.say("case: workspace blocks per stream")
    cfg = CONFIGS["cap20k"]
    xyz_t = make_positions(cfg)
    xyz = xyz_t.numpy()
    x = make_values(cfg, xyz_t).numpy()
    idx = G.build(xyz, x, cfg.edges_chord2())
    # on the current stream: (4, fp64) takes a block, (4, mixed) reuses it, (8, fp64) needs
    # more and replaces it, (8, mixed) reuses the larger one
    ref = {}
    for M in (4, 8):
        for prec in ("fp64", "mixed"):
            ref[(M, prec)] = z3.estimate(idx, M, prec=prec)
    other = torch.cuda.Stream()
    for stream in (other, torch.cuda.current_stream(), other):
        with torch.cuda.stream(stream):
            for M, prec in ((8, "fp64"), (4, "mixed"), (8, "mixed"), (4, "fp64")):
                z, pairs = z3.estimate(idx, M, prec=prec)
                zr, pr = ref[(M, prec)]
                assert pairs == pr, (M, prec)
                assert np.array_equal(z, zr), (M, prec)
    torch.cuda.synchronize()
    idx.free()
