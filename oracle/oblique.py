"""Textbook oblique-shock relations for a calorically perfect gas -- TEST
INFRASTRUCTURE ONLY (the exact reference for the oblique-shock checks of
Sec. V.F; the GPU library never imports it).

theta-beta-Mach relation (weak solution) and the Rankine-Hugoniot jumps of the
normal component, written from the standard gas-dynamics derivation:
    tan(theta) = 2 cot(beta) (M1^2 sin^2(beta) - 1) / (M1^2 (gamma + cos 2 beta) + 2)
    Mn1 = M1 sin(beta)
    rho2/rho1 = (gamma + 1) Mn1^2 / ((gamma - 1) Mn1^2 + 2)
    p2/p1     = 1 + 2 gamma / (gamma + 1) (Mn1^2 - 1)
    T2/T1     = (p2/p1) / (rho2/rho1)
    Mn2^2     = (1 + (gamma - 1)/2 Mn1^2) / (gamma Mn1^2 - (gamma - 1)/2)
    M2        = Mn2 / sin(beta - theta)
"""
import numpy as np
from scipy.optimize import brentq


def deflection(beta, mach, gamma=1.4):
    """Flow deflection theta (radians) behind an oblique shock of angle beta."""
    m2s = (mach * np.sin(beta)) ** 2
    return np.arctan(2.0 / np.tan(beta) * (m2s - 1.0) / (mach ** 2 * (gamma + np.cos(2 * beta)) + 2.0))


def weak_beta(mach, theta, gamma=1.4):
    """Weak-solution shock angle (radians) for deflection theta (radians)."""
    mu = np.arcsin(1.0 / mach)
    # the deflection rises from 0 at the Mach angle to its maximum, then falls
    bs = np.linspace(mu + 1e-9, np.pi / 2 - 1e-9, 20001)
    th = deflection(bs, mach, gamma)
    k = int(np.argmax(th))
    if theta > th[k]:
        raise ValueError("detached shock: theta above the maximum deflection")
    return brentq(lambda b: deflection(b, mach, gamma) - theta, mu + 1e-12, bs[k])


def jumps(mach, beta, theta, gamma=1.4):
    """(M2, rho2/rho1, T2/T1, p2/p1) behind the shock."""
    mn1 = mach * np.sin(beta)
    r = (gamma + 1.0) * mn1 ** 2 / ((gamma - 1.0) * mn1 ** 2 + 2.0)
    p = 1.0 + 2.0 * gamma / (gamma + 1.0) * (mn1 ** 2 - 1.0)
    mn2 = np.sqrt((1.0 + 0.5 * (gamma - 1.0) * mn1 ** 2) / (gamma * mn1 ** 2 - 0.5 * (gamma - 1.0)))
    m2 = mn2 / np.sin(beta - theta)
    return m2, r, p / r, p
