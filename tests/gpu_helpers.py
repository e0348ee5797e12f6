"""Shared helpers for the GPU tests (host-side marshalling and error metrics)."""
import numpy as np
import torch

from paper_2110_13042_amd import ata


def device():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU; none is visible")
    return torch.device("cuda:0")


def run_gram(A_np, mode, handle=None, lda=None):
    """Packed lower C from the HIP path (numpy FP64), A given on the host.

    For the FP32-family modes A must hold FP32 values (an FP32 array, or an
    FP64 array whose values are exact in FP32): the oracle the result is
    compared with then sees exactly the input the GPU sees.
    """
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    if mode != ata.F64 and np.asarray(A_np).dtype != np.float32:
        if not np.array_equal(np.asarray(A_np).astype(np.float32), A_np):
            raise ValueError("FP32-family input holds values that FP32 cannot represent; round it "
                             "to FP32 first so that the oracle sees the GPU's input")
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev, dt)
    if lda is not None and lda > A.shape[1]:
        big = torch.zeros((A.shape[0], lda), dtype=dt, device=dev)
        big[:, : A.shape[1]] = A
        A = big[:, : A_np.shape[1]]
    h = handle or ata.Handle()
    out = ata.gram(A, mode, handle=h)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def mode_input(A_np, mode):
    """A rounded to the element type the mode takes (FP64 for ATA_F64, else FP32)."""
    return np.asarray(A_np, dtype=np.float64 if mode == ata.F64 else np.float32)


def full_error(Cp, ref):
    """||C_hat - C||_F / ||C||_F over the full symmetric matrix (packed inputs)."""
    n = int((np.sqrt(8 * len(ref) + 1) - 1) / 2)
    diag = np.zeros(len(ref), dtype=bool)
    idx = np.arange(n)
    diag[idx * (idx + 1) // 2 + idx] = True
    w = np.where(diag, 1.0, 2.0)
    d = (Cp - ref) ** 2 * w
    return float(np.sqrt(d.sum() / (ref ** 2 * w).sum()))


def packed_columns(Cp, n, S):
    """Full columns C[:, S] (n x len(S)) from packed lower storage."""
    S = np.asarray(S)
    i = np.arange(n)[:, None]
    j = S[None, :]
    r, c = np.maximum(i, j), np.minimum(i, j)
    return Cp[r * (r + 1) // 2 + c]
