"""Shared helpers of the test suite (no method arithmetic: comparison metrics only)."""
import numpy as np


def full_from_packed(Cp, T):
    """[..., T(T+1)/2] -> symmetric [..., T, T]."""
    C = np.zeros(Cp.shape[:-1] + (T, T), dtype=np.float64)
    iu = np.triu_indices(T)
    C[..., iu[0], iu[1]] = Cp
    C[..., iu[1], iu[0]] = Cp
    return C


def eps_metric(C_test, C_ref):
    """|dC^{ij}| / sqrt(C^{ii} C^{jj}) of the reference, on full [L, T, T] matrices."""
    d = np.sqrt(np.abs(np.einsum("ltt->lt", C_ref)))
    den = d[:, :, None] * d[:, None, :]
    return np.abs(C_test - C_ref) / np.where(den > 0, den, 1.0)


def row_rel(W_test, W_ref):
    """max_j |dW| / max_j |W_ref| for every (l, t) row."""
    num = np.max(np.abs(W_test - W_ref), axis=-1)
    den = np.max(np.abs(W_ref), axis=-1)
    return num / np.where(den > 0, den, 1.0)
