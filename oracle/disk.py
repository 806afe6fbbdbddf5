"""Closed-form scattered field of a homogeneous disk.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 1, eq. (Helmholtz): (Delta + omega^2 (1 + m)) (u + u_I) = 0
with u outgoing (Sommerfeld).  For m = m0 on a disk of radius a (and 0
outside) and u_I = exp(i omega x) the separation of variables gives, with
k = omega sqrt(1 + m0) and polar coordinates (r, phi) about the disk centre,

  outside: u = sum_n c_n H_n(omega r) e^{i n phi}
  inside:  u = sum_n (b_n J_n(k r) - i^n J_n(omega r)) e^{i n phi}

where continuity of the total field and of its radial derivative at r = a
gives
  c_n = i^n [omega J_n'(omega a) J_n(k a) - k J_n(omega a) J_n'(k a)]
            / [k H_n(omega a) J_n'(k a) - omega H_n'(omega a) J_n(k a)],
  b_n = (i^n J_n(omega a) + c_n H_n(omega a)) / J_n(k a),
all times the phase exp(i omega x_c) of u_I at the centre.
This is the continuous solution; the discrete Lippmann-Schwinger solution
approaches it as h -> 0 (the jump of m limits the order).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def disk_scattered_field(X, Z, omega, contrast, radius, centre=(0.5, 0.5), nmax=None):
    k = omega * np.sqrt(1.0 + contrast)
    a = radius
    dx, dz = X - centre[0], Z - centre[1]
    r = np.sqrt(dx * dx + dz * dz)
    phi = np.arctan2(dz, dx)
    if nmax is None:
        nmax = int(1.5 * k * a) + 25
    u = np.zeros(X.shape, dtype=complex)
    inside = r <= a
    for nn in range(-nmax, nmax + 1):
        ina = 1j**nn
        Jwa, Jka = sp.jv(nn, omega * a), sp.jv(nn, k * a)
        dJwa, dJka = sp.jvp(nn, omega * a), sp.jvp(nn, k * a)
        Hwa, dHwa = sp.hankel1(nn, omega * a), sp.h1vp(nn, omega * a)
        c = ina * (omega * dJwa * Jka - k * Jwa * dJka) / (k * Hwa * dJka - omega * dHwa * Jka)
        b = (ina * Jwa + c * Hwa) / Jka
        e = np.exp(1j * nn * phi)
        u[~inside] += c * sp.hankel1(nn, omega * r[~inside]) * e[~inside]
        u[inside] += (b * sp.jv(nn, k * r[inside]) - ina * sp.jv(nn, omega * r[inside])) * e[inside]
    return u * np.exp(1j * omega * centre[0])
