"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np


def trainer_for(g, **kw):
    from paper_2604_09419_amd import Trainer
    return Trainer(g.n, g.src, g.dst, g.w, **kw)


def max_row_rel_err(x, ref):
    """max over rows r of ||x_r - ref_r|| / ||ref_r|| (rows with zero reference norm skipped)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    ok = den > 0
    return float(np.max(num[ok] / den[ok]))


def fro_rel_err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def dot_rows(A, B, u, v):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return np.einsum("ij,ij->i", A[u], B[v])
