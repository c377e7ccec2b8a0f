"""Shared helpers of the GPU tests (no method arithmetic here)."""
import numpy as np

KAPPA, CSW = 0.1394, 1.69
MU, MUBAR, EPSBAR = 0.01, 0.1246, 0.1315


def rel_l2(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)).cuda()


def to_host(t, shape):
    return t.cpu().numpy().reshape(shape)


def oracle_T_to_blocks(T):
    """Oracle clover [V][12][12] (index 3*spin+colour) -> [V][2][6][6] chirality blocks."""
    V = T.shape[0]
    out = np.empty((V, 2, 6, 6), dtype=np.complex128)
    for c in range(2):
        idx = np.arange(6 * c, 6 * c + 6)
        out[:, c] = T[:, idx][:, :, idx]
    return out
