"""Helpers of the GPU tests: run the HIP library through the C ABI on torch device
buffers and compare with the oracle by the per-field relative max-norm metric."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_bunch(layout, gamma, precision=8, **kw):
    from paper_2508_09568_amd.binding import Bunch
    return Bunch(layout.dims, g=layout.g, precision=precision, gamma=gamma, **kw)


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def field_scales(den):
    """Natural scale of each conserved component in a state with max-norms `den`:
    mass ||rho||, momentum sqrt(||rho|| ||E||), energy ||E||, field sqrt(||E||)."""
    r, e = den[0], den[4]
    nat = np.array([r, np.sqrt(r * e), np.sqrt(r * e), np.sqrt(r * e), e,
                    np.sqrt(e), np.sqrt(e), np.sqrt(e)])
    return np.maximum(den, nat)


def rel_err_fields(layout, A, B, patches=None):
    """Per-step parity metric: max over owned cells/faces of |A_f - B_f| divided by
    max(||B_f||_inf, natural scale of component f) (see field_scales).  Equal to the
    plain per-field relative max-norm whenever every field is of its natural size; a
    field that vanishes, or sits at noise level, is measured against the size the
    update's arithmetic works at."""
    patches = range(layout.P) if patches is None else patches
    num = np.zeros(8)
    den = np.zeros(8)
    for p in patches:
        a = layout.interior(A, p)
        b = layout.interior(B, p)
        num = np.maximum(num, np.abs(a - b).reshape(8, -1).max(axis=1))
        den = np.maximum(den, np.abs(b).reshape(8, -1).max(axis=1))
    return num / field_scales(den)


def plain_rel_err_fields(layout, A, B):
    """max over owned entries of |A_f - B_f| / ||B_f||_inf per field (no floor; a field
    that is identically zero in B reports its absolute difference)."""
    num = np.zeros(8)
    den = np.zeros(8)
    for p in range(layout.P):
        a = layout.interior(A, p)
        b = layout.interior(B, p)
        num = np.maximum(num, np.abs(a - b).reshape(8, -1).max(axis=1))
        den = np.maximum(den, np.abs(b).reshape(8, -1).max(axis=1))
    return num / np.where(den > 0, den, 1.0)


def l1_rel_fields(layout, A, B):
    num = np.zeros(8)
    den = np.zeros(8)
    for p in range(layout.P):
        a = layout.interior(A, p)
        b = layout.interior(B, p)
        num += np.abs(a - b).reshape(8, -1).sum(axis=1)
        den += np.abs(b).reshape(8, -1).sum(axis=1)
    den = np.where(den > 0, den, den[4])
    return num / den


def l1_rel_face_field(layout, A, B):
    """L1 difference of each face-field component (Bx, By, Bz) divided by the L1 magnitude of
    the whole face field, sum of |Bx| + |By| + |Bz| over owned faces."""
    num = np.zeros(3)
    den = 0.0
    for p in range(layout.P):
        a = layout.interior(A, p).reshape(8, -1)[5:]
        b = layout.interior(B, p).reshape(8, -1)[5:]
        num += np.abs(a - b).sum(axis=1)
        den += np.abs(b).sum()
    return num / den
