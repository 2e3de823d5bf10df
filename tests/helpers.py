"""Shared helpers for the GPU parity tests (HIP path through the C ABI)."""
from __future__ import annotations

import contextlib

import numpy as np


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@contextlib.contextmanager
def gpu_context(sys_, **overrides):
    """Creates an mdx context for a synth.System on cuda:0 and yields
    (mdx module, ctx handle, device tensors dict)."""
    import torch
    import paper_2503_20541_amd as mdx
    dev = torch.device("cuda:0")
    desc, keep = mdx.desc_from_system(sys_, **overrides)
    ctx = mdx.create(desc, torch.cuda.current_stream(dev).cuda_stream)
    t = dict(pos=torch.from_numpy(np.ascontiguousarray(sys_.pos)).to(dev),
             vel=torch.from_numpy(np.ascontiguousarray(sys_.vel)).to(dev),
             force=torch.zeros((3, sys_.n_atoms), dtype=torch.float32, device=dev),
             e_nb=torch.zeros(6, dtype=torch.float64, device=dev),
             e_rec=torch.zeros(1, dtype=torch.float64, device=dev))
    try:
        yield mdx, ctx, t
    finally:
        torch.cuda.synchronize()
        mdx.destroy(ctx)


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
