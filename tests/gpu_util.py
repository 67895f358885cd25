"""Helpers shared by the GPU parity tests (comparison metrics, padded device copies)."""
import numpy as np


def rel_l1(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def cosine(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def report(tag, gpu, ref):
    """Print the error of a GPU result against the FP64 oracle (shown with pytest -s / -v)."""
    e = rel_l1(gpu, ref)
    c = cosine(gpu, ref)
    print(f"[parity] {tag}: rel_l1={e:.3e} cos={c:.12f}", flush=True)
    return e, c


def to_dev(arr, torch_dtype=None, align_elems=None):
    """Copy a 1-D or 2-D numpy array to the GPU; 2-D rows are padded to a 16-byte pitch."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if torch_dtype is not None:
        t = t.view(torch_dtype) if t.element_size() == torch.empty(0, dtype=torch_dtype).element_size() else t.to(torch_dtype)
    if t.dim() == 2:
        n, m = t.shape
        es = t.element_size()
        per = 16 // es
        ld = (m + per - 1) // per * per
        buf = torch.zeros((n, ld), dtype=t.dtype, device="cuda")
        buf[:, :m] = t.cuda()
        return buf[:, :m]
    return t.cuda()
