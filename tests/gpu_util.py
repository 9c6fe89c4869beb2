"""Helpers shared by the GPU tests: library loading and the parity norm."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1907_08492_amd as P  # raises ImportError if libsipg.so is missing
    return torch, P


def rel_errors(y, ref):
    """(||y - ref||_2 / ||ref||_2, max|y - ref| / max|ref|)."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = y - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def banner(msg):
    print(f"[case] {msg}", flush=True)
