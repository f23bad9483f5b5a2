"""Helpers shared by the GPU tests (device copies, error norms)."""
import numpy as np


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel_linf(g, o, b):
    """Per-variable max |g - o| / max |o| over interior cells."""
    I = b.interior()
    d = np.abs(g[I] - o[I]).reshape(g.shape[0], -1).max(axis=1)
    s = np.abs(o[I]).reshape(o.shape[0], -1).max(axis=1)
    return d / np.where(s > 0, s, 1.0)


def norm_l1(g, o, b):
    I = b.interior()
    d = np.abs(g[I] - o[I]).reshape(g.shape[0], -1).sum(axis=1)
    s = np.abs(o[I]).reshape(o.shape[0], -1).sum(axis=1)
    return d / np.where(s > 0, s, 1.0)


def worst_cell(g, o, b):
    I = b.interior()
    d = np.abs(g[I] - o[I])
    idx = np.unravel_index(np.argmax(d), d.shape)
    return idx, g[I][idx], o[I][idx]


def padded_view(U, pad=(3, 1, 2)):
    """A copy of the device array U inside a larger NaN-filled array (pad =
    extra x elements per row, rows per plane, planes per variable): returns
    (storage, strided view of U's shape)."""
    import torch
    nv, NZ, NY, NX = U.shape
    big = torch.full((nv, NZ + pad[2], NY + pad[1], NX + pad[0]), float("nan"), dtype=U.dtype, device=U.device)
    view = big[:, :NZ, :NY, :NX]
    view.copy_(U)
    return big, view
