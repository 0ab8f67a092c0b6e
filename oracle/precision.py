"""FP32-data model of the linear step (test infrastructure only).

The precision extension (not part of the paper) runs the bulk of the ADMM
iterations with A and G^{-1} = (I + A A^T)^{-1} read from FP32 copies while all
arithmetic, the iterate, the border of the Schur reduction and the tests stay in
FP64.  ``Fp32DataSchurSolver`` is (I+Q)^{-1} w evaluated that way, so that the
GPU's FP32-data iterations can be compared with the oracle element by element
(to FP64 rounding) instead of only to the FP32 distance from the exact step.

It is the Schur / Sherman-Morrison-Woodbury solve of Section 4.4 (see
``oracle.abip.SchurIQSolver``) with three data choices written out:
  * t = w_y - fl(A) w_x and a = fl(G^{-1}) t, where fl rounds to FP32;
  * d = w_x + fl(A)^T a;
  * the border terms use c^T d = c^T w_x + (A c)^T a and
    cbar^T d = cbar^T w_x + (A cbar)^T a with the FP64 products A c, A cbar
    (the same real numbers as c^T d and cbar^T d in exact data), and the FP64
    border Z = M^{-1} H and 2 x 2 K of the exact data.
With ``dtype=np.float64`` nothing is rounded and the result equals the exact
Schur solve up to rounding order (pinned in tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .abip import SchurIQSolver, hsd_constants


class Fp32DataSchurSolver:
    def __init__(self, prob, dtype=np.float32):
        A = prob.A
        m, n = A.shape
        self.m, self.n = m, n
        self.b = prob.b
        self.c = prob.c
        bbar, cbar, _ = hsd_constants(prob)
        self.bbar, self.cbar = bbar, cbar
        G = np.eye(m) + A @ A.T
        Ginv = sla.cho_solve(sla.cho_factor(G, lower=True), np.eye(m))
        Ginv = 0.5 * (Ginv + Ginv.T)
        self.Ar = A.astype(dtype).astype(np.float64)
        self.Gr = Ginv.astype(dtype).astype(np.float64)
        self.Ac = A @ prob.c
        self.Acb = A @ cbar
        exact = SchurIQSolver(prob)
        self.Z = exact.Z
        self.Kinv = np.linalg.inv(exact.K)

    def solve(self, w):
        m, n = self.m, self.n
        y, f = w[:m], w[m:m + n]
        t = y - self.Ar @ f
        a = self.Gr @ t
        d = f + self.Ar.T @ a
        h1z = -(self.b @ a) + (self.c @ f) + (self.Ac @ a)
        h2z = (self.bbar @ a) - (self.cbar @ f) - (self.Acb @ a)
        p = self.Kinv @ (w[m + n:] + np.array([h1z, h2z]))
        z = np.concatenate([a, d])
        return np.concatenate([z - self.Z @ p, p])
