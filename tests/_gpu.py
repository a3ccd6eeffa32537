"""Helpers of the GPU tests: device transfer and the library calls."""
import sys

import numpy as np
import pytest
import torch

from paper_1303_5837_amd import caqr


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this host")


def banner(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tsqr_gpu(A, **kw):
    dA = caqr.fortran(A)
    F = caqr.tsqr(dA, **kw)
    torch.cuda.synchronize()
    return F, F.R.cpu().numpy()


def caqr_gpu(A, nb=64, **kw):
    dA = caqr.fortran(A)
    F = caqr.caqr(dA, nb=nb, **kw)
    torch.cuda.synchronize()
    return F, F.R.cpu().numpy()


def factored(F):
    return F.A.cpu().numpy()


def q_thin(F):
    Q = F.q_thin()
    torch.cuda.synchronize()
    return Q.cpu().numpy()
