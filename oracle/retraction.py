"""Softplus retraction map (section 4.1, eq. softplus; appendix C).

b_kappa(v) maps R -> R_+ with b_kappa(v) * b_kappa(-v) = kappa (eq. retraction
map), so z = b_kappa(v), s = b_kappa(-v) satisfy z*s = kappa by construction.

Test infrastructure only (see package docstring).
"""
import numpy as np


def b_plain(v, kappa):
    """Definition: b_kappa(v) = (v + sqrt(v^2 + 4 kappa)) / 2  (eq. softplus).
    Loses all digits for v << 0; used only to pin the branch form."""
    v = np.asarray(v)
    return (v + np.sqrt(v * v + 4.0 * kappa)) / 2.0


def b(v, kappa):
    """Cancellation-free b_kappa(v) (appendix C): the definition for v >= 0,
    the conjugate form 2 kappa / (sqrt(v^2 + 4 kappa) - v) for v < 0."""
    v = np.asarray(v)
    r = np.sqrt(v * v + 4.0 * kappa)
    with np.errstate(divide="ignore", invalid="ignore"):
        neg = 2.0 * kappa / (r - v)
    return np.where(v >= 0, (v + r) / 2.0, neg)


def db_dv(v, kappa):
    """d b_kappa(v) / dv (appendix C): (1 + v/r)/2 for v >= 0 and
    2 kappa / (r^2 - v r) for v < 0, with r = sqrt(v^2 + 4 kappa).
    Properties (eq. softplus properties): db(v) + db(-v) = 1, 0 < db <= 1."""
    v = np.asarray(v)
    r = np.sqrt(v * v + 4.0 * kappa)
    with np.errstate(divide="ignore", invalid="ignore"):
        neg = 2.0 * kappa / (r * r - v * r)
    return np.where(v >= 0, 0.5 * (1.0 + v / r), neg)


def db_dkappa(v, kappa):
    """c = d b_kappa(v) / d kappa = 1 / sqrt(v^2 + 4 kappa); the same value
    for b_kappa(-v) (section 4.2, below eq. implicit_kkt)."""
    v = np.asarray(v)
    return 1.0 / np.sqrt(v * v + 4.0 * kappa)
