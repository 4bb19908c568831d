"""Continuous colour and polarization sampling with the dressed recursion
(Section 2.1, eqs. polarization_kleiss, polarization_axial,
polarization_simple, color_angles, gluon_color_polarization; the paper's
colour-dressed sampled variant of Section 3).  TEST INFRASTRUCTURE.

Polarization: with the external currents X^h = (eps^h)* of
``polarization`` (X^+ = (e1 - i e2)/sqrt2, X^- = (X^+)*), the vector
    e(phi) = e^{i phi} X^+ + e^{-i phi} X^- = sqrt2 (cos phi e1 + sin phi e2)
is real, and averaging e_mu e_nu over phi uniform in [0, 2 pi) gives
sum_h X^h_mu X^h*_nu, so the phi-average of |A(e(phi))|^2 is the helicity
sum (each amplitude is linear in each polarization).  Reading: the paper
writes the same vector with differently normalised e1, e2; the factor sqrt2
is the one that makes the average the helicity sum for these currents.

Colour: a gluon carries two real unit vectors eta = eta(z), etabar =
eta(zbar), uniform on the sphere (eq. color_angles).  Its colour
wavefunction eta^a = eta T^a etabar, contracted into the trace basis with
sum_a T^a_kl T^a_ij = d_il d_kj - d_kl d_ij / N, acts as the 3x3 matrix
etabar eta^T (row from zbar, column from z) minus a multiple of the unit
matrix, which decouples from pure-gluon amplitudes.  So the amplitude is the
dressed recursion with external colour matrices etabar_k eta_k^T in place of
the colour-flow matrices e_{j_k i_k}, closed with eta_n^T M etabar_n; a flow
assignment (i_k, j_k) is the special case eta = e_{i_k}, etabar = e_{j_k}.
With the measure of the paper each of the two sphere integrals per gluon is
N_c times the uniform average, so
    sum over colours and helicities of |M|^2 = 9^n E[A^2]
for phi_k uniform and eta, etabar uniform on the unit sphere.  With real
polarizations and colour vectors every current and the amplitude are real.

Arrays: phi [n][E]; eta [2][n][3][E] with eta[0][k] = eta(z_k) and
eta[1][k] = eta(zbar_k).
"""
import math

import numpy as np

from .cdbg import dressed_recursion
from .cobg import G_S, momenta_list
from .lorentz import mdot
from .numeric import sqrt2
from .polarization import basis

NC = 3
COLOUR_WEIGHT = NC * NC  # per gluon: two sphere integrals of N_c times the average


def real_polarizations(ps, phi):
    """e_k(phi_k) = sqrt2 (cos phi_k e1(p_k) + sin phi_k e2(p_k)): list of [4][E]."""
    out = []
    for k, p in enumerate(ps):
        e1, e2 = basis(p)
        c, s = np.cos(phi[k]), np.sin(phi[k])
        out.append([sqrt2(p[0]) * (c * e1[m] + s * e2[m]) for m in range(4)])
    return out


def colour_matrices(eta):
    """etabar_k eta_k^T per gluon: list of [3,3,E]."""
    n = eta.shape[1]
    return [eta[1, k][:, None, :] * eta[0, k][None, :, :] for k in range(n)]


def amplitude_general(ps, eps, colmats, eta_n, etabar_n, g=None, tensor=True):
    """eta_n^T (eps_n . P^2 J(1..n-1)) etabar_n for given external currents and
    colour matrices of gluons 1..n-1: complex [E]."""
    n = len(ps)
    J = dressed_recursion(ps, eps[: n - 1], colmats[: n - 1], g=g, tensor=tensor)
    top = J[(1 << (n - 1)) - 1]  # [3,3,4,E]
    m = mdot(eps[n - 1], [top[:, :, mu, :] for mu in range(4)])  # [3,3,E]
    return np.einsum("ae,abe,be->e", eta_n, m, etabar_n)


def continuous_amplitude(mom, phi, eta, g=None, tensor=True):
    """Amplitude for real polarizations e(phi) and colour vectors eta: complex
    [E] whose imaginary part vanishes (kept for the reality check)."""
    ps = momenta_list(mom)
    eps = real_polarizations(ps, phi)
    n = mom.shape[0]
    return amplitude_general(ps, eps, colour_matrices(eta), eta[0, n - 1], eta[1, n - 1],
                             g=g, tensor=tensor)


def me2_continuous(mom, phi, eta, g=None, tensor=True):
    """A^2 per event (float [E]); 9^n times its mean is the colour- and
    helicity-summed |M|^2."""
    a = continuous_amplitude(mom, phi, eta, g=g, tensor=tensor)
    return np.real(a) ** 2


def sphere_vector(u_cos, u_phi):
    """eta(theta, phi) of eq. color_angles with cos theta = 2 u_cos - 1 and
    phi = 2 pi u_phi: [3] + shape of the inputs."""
    c = 2.0 * np.asarray(u_cos) - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    ph = 2.0 * np.pi * np.asarray(u_phi)
    return np.stack([c, s * np.cos(ph), s * np.sin(ph)])
