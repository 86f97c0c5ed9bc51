"""Helpers shared by the GPU tests (loading the built library, moving data)."""

import os

import numpy as np
import torch


def tm():
    import paper_1807_11313_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1807_11313_amd import build
        build.build()
    pkg.lib()
    return pkg


def dev(x, dtype=None):
    t = torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x)
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def banner(msg):
    print("[gpu] " + msg, flush=True)
