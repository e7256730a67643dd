"""Helpers shared by the GPU tests (no method arithmetic beyond reading the
documented factor layout)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# Relative error allowed above the stopping bound of a mixed solve: the bound (ADI lemma,
# Sec. 5.1) covers the truncation error of the rounds in exact arithmetic, not FP64
# rounding (of the solve, and of the test's own G0 = A U0, whose rounding moves the exact
# solution by up to the condition number times the unit roundoff).  The largest excess
# measured is 7e-12, on Neumann problems with omega^2 <= 0.05 (spectral ratios 1e10-1e13).
ROUNDING_ALLOWANCE = 2e-11


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def structured_to_dense(buf, n, p, bc):
    """Dense lower-triangular L from the structured factor record documented in
    include/hpadi.h (hpadi_plan_export_factor)."""
    nh = n - 1 if bc == "dirichlet" else n + 1
    N = nh + n * (p - 1)
    nb = (p - 1) * n
    invd, link = buf[:nb], buf[nb:2 * nb]
    cpl = buf[2 * nb:2 * nb + 4 * n]
    invd0 = buf[2 * nb + 4 * n:2 * nb + 4 * n + nh]
    link0 = buf[2 * nb + 4 * n + nh:2 * nb + 4 * n + 2 * nh]
    L = np.zeros((N, N))
    for h in range(nh):
        L[h, h] = 1.0 / invd0[h]
        if h > 0:
            L[h, h - 1] = link0[h]

    def hat(v):
        if bc == "dirichlet":
            return v - 1 if 1 <= v <= n - 1 else None
        return v
    for m in range(p - 1):
        for e in range(n):
            r = nh + m * n + e
            L[r, r] = 1.0 / invd[m * n + e]
            if m >= 2:
                L[r, r - 2 * n] = link[m * n + e]
            if m <= 1:
                for side, v in ((0, e), (1, e + 1)):
                    hv = hat(v)
                    if hv is not None:
                        L[r, hv] = cpl[4 * e + 2 * m + side]
    return L


def factor_len(n, p, bc):
    nh = n - 1 if bc == "dirichlet" else n + 1
    return 2 * (p - 1) * n + 4 * n + 2 * nh
