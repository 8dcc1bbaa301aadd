"""Helpers shared by the GPU parity tests (comparison metrics only)."""
import numpy as np
import torch

DEV = "cuda:0"


def rel_err_rows(got, ref):
    """Per-row relative error |got_i - ref_i| / |ref_i| (Euclidean norms)."""
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape)
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return num / np.where(den > 0, den, 1.0)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()
