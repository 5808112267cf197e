"""Helpers shared by the GPU tests: host<->device copies and the tolerance
metric (per column: ||y - y_ref||_2 / ||y_ref||_2, worst column)."""

import numpy as np

TOL = {"c64": 2e-5, "c128": 1e-12}


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(y, ref):
    y = np.atleast_2d(np.asarray(y, dtype=np.complex128))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.complex128))
    num = np.linalg.norm(y - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return float(np.max(num / den))


def crandn(rng, shape, dtype=np.complex64):
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) * np.sqrt(0.5)).astype(dtype)
