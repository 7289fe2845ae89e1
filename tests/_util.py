"""Helpers shared by the tests (no method arithmetic here)."""
import numpy as np


def rms_err(a, ref):
    """max_b |a_b - ref_b| / rms_b |ref_b| over a batch (amplitude error metric)."""
    a = np.asarray(a)
    ref = np.asarray(ref)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    if scale == 0:
        return float(np.max(np.abs(a - ref)))
    return float(np.max(np.abs(a - ref)) / scale)


def gpu_amplitudes(plan, bitstrings, slice_range=None, repeat=1):
    """Run qx_contract on the current stream and return complex128 amplitudes on the host."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64)).view(np.int64)).cuda()
    amp = torch.zeros((len(bitstrings), 2), dtype=torch.float64, device="cuda")
    for _ in range(repeat):
        plan.contract(x, amp, slice_range)
    torch.cuda.synchronize()
    h = amp.cpu().numpy()
    return h[:, 0] + 1j * h[:, 1]
