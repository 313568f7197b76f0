"""The same two-stream equations as oracle/two_stream.py solved by a
different algorithm, used only to pin that oracle: closed-form reflection
and transmission of each homogeneous layer (the source-free modes
exp(+-k tau) plus the particular solution of the direct beam), combined
through the column with the adding method.  Near the resonance k mu0 = 1,
where the particular solution is singular, a layer's direct-beam terms are
the mean of their values at mu0 (1 -+ 1e-5): an O(1e-10) error from the
mean, O(1e-11) from cancellation just outside the window.

The PIFM coefficients and equations are those stated in
oracle/two_stream.py (Zdunkowski, Welch and Korb 1980; Meador and Weaver
1980, Table 1)."""
from __future__ import annotations

import numpy as np

K_MIN = 1e-12          # floor of the eigenvalue k (conservative scattering)
RESONANCE = 1e-5       # |1 - k^2 mu0^2| below this: resonant layer
DELTA = 1e-5           # relative shift of mu0 around a resonance


def gammas(ssa, g, mu0):
    """PIFM coefficients (gamma1, gamma2, gamma3, gamma4)."""
    ssa = np.asarray(ssa, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    return (8.0 - ssa * (5.0 + 3.0 * g)) / 4.0, 3.0 * ssa * (1.0 - g) / 4.0, \
        (2.0 - 3.0 * mu0 * g) / 4.0, (2.0 + 3.0 * mu0 * g) / 4.0


def layer(tau, ssa, g, mu0):
    """Reflection and transmission of one homogeneous layer.

    Returns (R, T, Rdir, Tdir, Tb):
      R, T     diffuse reflectance and transmittance for diffuse light on
               either face (the layer is symmetric for diffuse light);
      Rdir     upward diffuse flux at the top, Tdir downward diffuse flux at
               the bottom, per unit direct horizontal flux at the top;
      Tb       exp(-tau/mu0), the unscattered direct transmittance.
    """
    g1, g2, g3, g4 = gammas(ssa, g, mu0)
    k = np.sqrt(np.maximum((g1 - g2) * (g1 + g2), 0.0))
    k = np.maximum(k, K_MIN)
    # homogeneous problem (no direct beam): modes exp(+-k tau); with
    # E = exp(-k tau) and X = 1 - E^2 the two-point problem gives
    E = np.exp(-k * tau)
    X = -np.expm1(-2.0 * k * tau)
    den = k * (1.0 + E * E) + g1 * X
    R = g2 * X / den
    T = 2.0 * k * E / den
    Rdir, Tdir = _direct(tau, ssa, g1, g2, g3, g4, k, R, T, mu0)
    # the particular solution is singular where k mu0 = 1 although Rdir and
    # Tdir are smooth there: near that resonance they are the mean of their
    # values at mu0 (1 - DELTA) and mu0 (1 + DELTA) (error O(DELTA^2), no
    # division by a small number)
    near = np.abs(1.0 - k * k * mu0 * mu0) < RESONANCE
    if np.any(near):
        both = []
        for m in (mu0 * (1.0 - DELTA), mu0 * (1.0 + DELTA)):
            _, _, h3, h4 = gammas(ssa, g, m)
            both.append(_direct(tau, ssa, g1, g2, h3, h4, k, R, T, m))
        Rdir = np.where(near, 0.5 * (both[0][0] + both[1][0]), Rdir)
        Tdir = np.where(near, 0.5 * (both[0][1] + both[1][1]), Tdir)
    Tb = np.exp(-tau / mu0)
    return R, T, Rdir, Tdir, Tb


def _direct(tau, ssa, g1, g2, g3, g4, k, R, T, mu0):
    """(Rdir, Tdir) of a layer for the sun at cosine mu0.  Particular
    solution for unit direct horizontal flux at the top (P0 = 1/mu0):
    U_p = a exp(-tau/mu0), D_p = b exp(-tau/mu0) with
      (gamma1 + 1/mu0) a - gamma2 b = gamma3 w P0,
      gamma2 a + (1/mu0 - gamma1) b = -gamma4 w P0;
    the homogeneous solution that cancels D at the top (-b) and U at the
    bottom (-a Tb) is, by the definition of R and T, R and T applied to
    those two incident fluxes."""
    d = 1.0 - k * k * mu0 * mu0
    a = ssa * (g3 * (1.0 - g1 * mu0) - g2 * g4 * mu0) / d
    b = -ssa * (g4 * (1.0 + g1 * mu0) + g2 * g3 * mu0) / d
    Tb = np.exp(-tau / mu0)
    return a - R * b - T * a * Tb, b * Tb - T * b - R * a * Tb


def column(tau, ssa, g, mu0, albedo, flux_toa=1.0):
    """Fluxes at the nlay+1 levels of a column of homogeneous layers.

    tau, ssa, g: [nlay], layer 0 at the TOA.  flux_toa: solar flux normal
    to the beam at the TOA, so the direct horizontal flux there is
    flux_toa * mu0.  Returns (direct, down_diffuse, up) [nlay+1], W m^-2 in
    the units of flux_toa; level 0 is the TOA, level nlay the surface.

    Adding method: sweeping up from the surface, Rb[i] is the diffuse albedo
    of everything below level i and Q[i] the upward diffuse flux at level i
    produced by the direct beam below level i (with no diffuse light coming
    down through level i); then sweeping down, the diffuse downward flux
    follows from multiple reflection between each layer and what lies below
    it, and U[i] = Rb[i] D[i] + Q[i].
    """
    tau = np.asarray(tau, dtype=np.float64)
    ssa = np.asarray(ssa, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = tau.size
    R, T, Rdir, Tdir, Tb = layer(tau, ssa, g, mu0)
    S = np.empty(n + 1)
    S[0] = flux_toa * mu0
    for l in range(n):
        S[l + 1] = S[l] * Tb[l]
    Rb = np.empty(n + 1)
    Q = np.empty(n + 1)
    Rb[n] = albedo
    Q[n] = albedo * S[n]
    for l in range(n - 1, -1, -1):
        m = 1.0 / (1.0 - R[l] * Rb[l + 1])
        Rb[l] = R[l] + T[l] * T[l] * Rb[l + 1] * m
        Q[l] = Rdir[l] * S[l] + T[l] * (Q[l + 1] + Rb[l + 1] * Tdir[l] * S[l]) * m
    D = np.empty(n + 1)
    D[0] = 0.0
    for l in range(n):
        D[l + 1] = (T[l] * D[l] + Tdir[l] * S[l] + R[l] * Q[l + 1]) / (1.0 - R[l] * Rb[l + 1])
    U = Rb * D + Q
    return S, D, U


def top_of_domain(tau, ssa, g, mu0, albedo, level, flux_toa=1.0):
    """(total downward flux, diffuse fraction) at level `level` of the
    column (the top of the ray tracer's domain)."""
    S, D, _ = column(tau, ssa, g, mu0, albedo, flux_toa)
    tot = S[level] + D[level]
    return tot, (D[level] / tot if tot > 0 else 0.0)
