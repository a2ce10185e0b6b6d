"""Helpers shared by the GPU tests: seeded inputs, dtype tolerances, errors."""
import sys

import numpy as np
import torch

from paper_2507_02420_amd.inputs import gaussian, haar_unitary

# normwise relative tolerance per storage dtype (FP64 1e-12, FP32 1e-5,
# BF16 1e-2; FP16 shares the BF16 bound; int32 is compared bit for bit)
TOL = {torch.float64: 1e-12, torch.complex128: 1e-12, torch.float32: 1e-5, torch.complex64: 1e-5,
       torch.bfloat16: 1e-2, torch.float16: 1e-2}
W_DT = {torch.float64: torch.float64, torch.float32: torch.float32, torch.complex128: torch.complex128,
        torch.complex64: torch.complex64, torch.bfloat16: torch.float32, torch.float16: torch.float32,
        torch.int32: torch.int32}
COMPLEX = (torch.complex64, torch.complex128)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_inputs(b, n, batch, dtype, seed, W=None):
    """Device x (batch, b**n) and W in the plan's dtypes, plus their exact
    float64/complex128 values as held on the device (for the oracle)."""
    cplx = dtype in COMPLEX
    x = gaussian((batch, b ** n), seed=seed, complex_=cplx)
    if W is None:
        W = haar_unitary(b, seed + 1, complex_=cplx)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dtype)
    Wt = torch.from_numpy(np.ascontiguousarray(W)).to(W_DT[dtype])
    x64 = xt.to(torch.complex128 if cplx else torch.float64).numpy()
    W64 = Wt.to(torch.complex128 if cplx else torch.float64).numpy()
    return xt.cuda(), Wt.cuda(), x64, W64


def host64(t):
    t = t.detach().cpu()
    if t.is_complex():
        return t.to(torch.complex128).numpy()
    return t.to(torch.float64).numpy()


def rel_err(y, ref):
    """Largest per-instance normwise relative error ||y - ref|| / ||ref||."""
    y = np.atleast_2d(y)
    ref = np.atleast_2d(ref)
    num = np.linalg.norm(y - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float(np.max(num / den))
