"""Preconditioned MINRES of Paige and Saunders (Section 6.1), x0 = 0.

Lanczos process in the M-inner product (M^{-1} = one V-cycle), the
tridiagonal least-squares problem solved by Givens rotations, and the
residual-norm estimate phi_bar = ||r_k||_{M^{-1}}.  Stopping test eq. (6.2)
||r|| <= eps ||b|| read in that same norm: phi_bar <= eps * beta_1 with
beta_1 = sqrt(b^T M^{-1} b).

A negative M-norm (r^T M^{-1} r < 0) means that the preconditioner is not
positive definite in floating point.  By default this raises NotSPD; with
stop_on_indefinite the iteration ends there and returns the iterate reached
before that Lanczos step (used by the interior point method, whose systems
become ill-conditioned enough for the V-cycle to lose definiteness).
"""
from __future__ import annotations

import math

import numpy as np


class NotSPD(RuntimeError):
    pass


def minres(A, b, Minv, eps, maxit, stop_on_indefinite=False):
    """Returns (x, iterations, phi_bar/beta_1)."""
    n = b.size
    x = np.zeros(n)
    r1 = b.copy()
    y = Minv(r1)
    beta1sq = float(r1 @ y)
    if beta1sq < 0:
        if stop_on_indefinite:
            return x, 0, 1.0
        raise NotSPD("preconditioner not positive definite")
    if beta1sq == 0:
        return x, 0, 0.0
    beta1 = math.sqrt(beta1sq)
    beta, beta_old = beta1, 0.0
    r2 = r1.copy()
    v_old = np.zeros(n)          # not needed beyond the recurrence
    w = np.zeros(n)
    w2 = np.zeros(n)
    c, s = -1.0, 0.0
    dbar, eps_l = 0.0, 0.0
    phibar = beta1
    it = 0
    for it in range(1, maxit + 1):
        v = y / beta                          # Lanczos vector (M-orthonormal)
        y = A(v)
        if it >= 2:
            y = y - (beta / beta_old) * r1
        alpha = float(v @ y)
        y = y - (alpha / beta) * r2
        r1, r2 = r2, y
        y = Minv(r2)
        beta_old = beta
        bsq = float(r2 @ y)
        if bsq < 0:
            if stop_on_indefinite:
                return x, it, phibar / beta1
            raise NotSPD("preconditioner not positive definite")
        beta = math.sqrt(bsq)
        # apply the previous rotation, then build the new one
        eps_old = eps_l
        delta = c * dbar + s * alpha
        gbar = s * dbar - c * alpha
        eps_l = s * beta
        dbar = -c * beta
        gamma = math.hypot(gbar, beta)
        gamma = max(gamma, np.finfo(float).eps)
        c, s = gbar / gamma, beta / gamma
        phi = c * phibar
        phibar = s * phibar
        w1, w2 = w2, w
        w = (v - eps_old * w1 - delta * w2) / gamma
        x = x + phi * w
        if phibar <= eps * beta1:
            break
    return x, it, phibar / beta1
