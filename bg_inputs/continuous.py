"""Continuous colour and polarization variables for the sampled variant with
real polarizations (Section 2.1, eqs. polarization_simple, color_angles).

Per event (counter e of the keyed SplitMix64 stream) and gluon k, five
uniforms in draw slots 5k .. 5k+4: the polarization angle phi_k = 2 pi u,
then (cos theta, azimuth) of eta(z_k) and of eta(zbar_k), each mapped to a
unit vector (cos theta, sin theta cos phi, sin theta sin phi) with
cos theta = 2u - 1 and phi = 2 pi u, i.e. uniform on the sphere.

Arrays: phi [n][E] float64, eta [2][n][3][E] float64 with eta[0][k] =
eta(z_k) and eta[1][k] = eta(zbar_k).
"""
import math

import numpy as np

from .rng import splitmix64_uniform


def _unit(u_cos, u_az):
    c = 2.0 * u_cos - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    a = 2.0 * math.pi * u_az
    return np.stack([c, s * np.cos(a), s * np.sin(a)])  # [3][E]


def continuous_states(n, n_events, seed, first=0):
    """(phi [n][E], eta [2][n][3][E]) for events first .. first+n_events-1 of
    stream seed."""
    ctr = np.arange(first, first + n_events, dtype=np.uint64)
    u = splitmix64_uniform(seed, ctr, 5 * n)  # [E, 5n]
    phi = np.empty((n, n_events))
    eta = np.empty((2, n, 3, n_events))
    for k in range(n):
        phi[k] = 2.0 * math.pi * u[:, 5 * k]
        eta[0, k] = _unit(u[:, 5 * k + 1], u[:, 5 * k + 2])
        eta[1, k] = _unit(u[:, 5 * k + 3], u[:, 5 * k + 4])
    return phi, eta
