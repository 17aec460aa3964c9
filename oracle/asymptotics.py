"""Thin-interface constants of the alloy phase-field model (Appendix A).

Test infrastructure (see the package docstring).

``closed_form`` writes out the constants the paper prints at the end of
Appendix A (solvability condition, the I, J, F, H, K integrals and the
values of a1, a2; the lambda' remark that gives a1' = 5 sqrt(2)/8 and
a2' = 47/75).  ``quadrature`` evaluates the same integrals from their
definitions over the leading-order profile psi_0(eta) of Appendix A with
plain trapezoidal sums; the tests compare the two.
"""
from __future__ import annotations

import math

import numpy as np


def closed_form(beta_psi=0.25, psi_s=1.0, psi_l=-1.0):
    """I, J, F, H, K, a1 = I/J, a2 = (K + J H)/I as printed in Appendix A."""
    dpsi = psi_s - psi_l
    r = math.sqrt(2.0 * beta_psi)
    I = r / 6.0 * dpsi ** 3
    J = 1.0
    F = 0.0
    H = math.log(2.0) / (r * dpsi)
    K = (47.0 / 60.0 - math.log(2.0)) / (r * dpsi)
    a1 = I / J
    a2 = (K + J * H) / I
    return dict(I=I, J=J, F=F, H=H, K=K, a1=a1, a2=a2)


def quadrature(beta_psi=0.25, psi_s=1.0, psi_l=-1.0, L=40.0, n=400001):
    """The same constants from their integral definitions (Appendix A).

    psi_0 is the leading-order inner solution (decreasing in eta, solid at
    eta -> -inf); h(psi) = (psi - psi_l)/(psi_s - psi_l); p'(psi) is the
    derivative of the interpolation function p of Sec. 2.1,
    30 (psi_s - psi)^2 (psi - psi_l)^2 / (psi_s - psi_l)^5.
    """
    dpsi = psi_s - psi_l
    r = math.sqrt(2.0 * beta_psi)
    eta = np.linspace(-L, L, n)
    de = eta[1] - eta[0]
    arg = 0.5 * dpsi * r * eta
    psi0 = 0.5 * (psi_s + psi_l) - 0.5 * dpsi * np.tanh(arg)
    dpsi0 = -0.5 * dpsi * 0.5 * dpsi * r / np.cosh(arg) ** 2
    h = (psi0 - psi_l) / dpsi
    pprime = 30.0 * (psi_s - psi0) ** 2 * (psi0 - psi_l) ** 2 / dpsi ** 5

    def trap(y):
        return float(np.sum(0.5 * (y[1:] + y[:-1])) * de)

    I = trap(dpsi0 ** 2)
    J = -trap(pprime * dpsi0)
    F = trap(eta * pprime * dpsi0)
    # int_0^eta h(psi_0) dzeta, cumulative from eta = 0 in both directions
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (h[1:] + h[:-1]) * de)])
    i0 = n // 2
    cum = cum - cum[i0]
    K = trap(pprime * dpsi0 * cum)
    # H^+ = int_0^inf [h(psi_0) - 0] d eta  (liquid side, h -> 0)
    Hp = trap(h[i0:])
    # H^- = int_0^-inf [h(psi_0) - 1] d eta  (solid side, h -> 1)
    Hm = -trap(h[: i0 + 1] - 1.0)
    a1 = I / J
    a2 = (K + J * Hp) / I
    return dict(I=I, J=J, F=F, H=Hp, Hminus=Hm, K=K, a1=a1, a2=a2)
