"""Helpers of the GPU tests."""
import numpy as np
import pytest


def require_gpu():
    try:
        import torch
        ok = torch.cuda.is_available()
    except Exception:
        ok = False
    if not ok:
        pytest.skip("no GPU")
    import paper_1202_4748_amd as lbf
    lbf.lib()  # fails loudly if the library is missing
    return lbf


def say(*a):
    print(*a, flush=True)


def rel_err(x, ref):
    """max |x - ref| / max |ref| (the field tolerance of the parity tests)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def dev_rel_err(rho, rho_ref):
    """Deviation-relative error || drho - drho_ref ||_2 / || drho_ref ||_2."""
    d = rho - rho_ref.mean()
    d_ref = rho_ref - rho_ref.mean()
    return float(np.linalg.norm(d - d_ref) / max(np.linalg.norm(d_ref), 1e-300))
