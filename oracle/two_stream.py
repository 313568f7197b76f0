"""FP64 oracle of the clear-sky two-stream column that sets the flux at the
top of the ray tracer's domain.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the smoke check,
never by the product path; it shares no code with the HIP implementation.

Sec. 2.3 (initialisation paragraph): before tracing, the total incoming
flux and its diffuse fraction at the top of the domain (TOD) come from a
two-stream calculation on a clear-sky 1D profile that spans surface to top
of atmosphere (TOA); photons then enter the domain along the sun beam or,
with the diffuse fraction, as isotropic downwelling radiation.  The paper
names only "a two-stream solver" (that of its host radiation package).
Readings taken here:

* two-stream coefficients: the practical improved flux method (PIFM) of
  Zdunkowski, Welch and Korb (1980), as tabulated by Meador and Weaver
  (1980, J. Atmos. Sci. 37, Table 1):
      gamma1 = (8 - w (5 + 3 g)) / 4,  gamma2 = 3 w (1 - g) / 4,
      gamma3 = (2 - 3 mu0 g) / 4,      gamma4 = 1 - gamma3;
* equations, tau increasing downward, U/D upward/downward diffuse flux,
  P = S / mu0 with S the direct horizontal flux:
      dU/dtau = gamma1 U - gamma2 D - gamma3 w P
      dD/dtau = gamma2 U - gamma1 D + gamma4 w P
      dP/dtau = -P / mu0;
* boundary conditions: at the TOA no diffuse light comes down (D = 0) and
  P = the flux normal to the beam; the surface is Lambertian with one
  albedo for direct and diffuse light, U = albedo (D + mu0 P);
* each layer is homogeneous; gas layers scatter with the Rayleigh phase
  function (g = 0).

The solution is the plain definition of that two-point boundary-value
problem: in a homogeneous layer y = (U, D, P) obeys dy/dtau = A y with a
constant matrix A, so y(tau0 + t) = expm(A t) y(tau0) exactly.  Every layer
is cut into equal sub-layers short enough that expm(A t) grows by at most
exp(1/2) (this changes nothing in exact arithmetic and keeps the system
well conditioned), and the transfer relations of all sub-layers plus the
three boundary conditions form one banded linear system for y at every
sub-level, solved with LAPACK's banded LU.  No closed-form layer solution,
no adding method and no special case at the resonance k mu0 = 1 (where
closed-form particular solutions are singular) are involved.

Parity pins (tests/test_two_stream_pins.py): Beer-Lambert and exp(-2 tau)
closed forms for a pure absorber, exact energy conservation for
conservative scattering, single-scattering backscatter of a thin layer by
quadrature of the phase function, the adding method with closed-form layer
coefficients (an independent algorithm), and exact Monte Carlo transport
within the approximation's known accuracy.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm, solve_banded

MAX_GROWTH = 0.5       # largest k * t of a sub-layer


def gammas(ssa, g, mu0):
    """PIFM coefficients (gamma1, gamma2, gamma3, gamma4)."""
    ssa = np.asarray(ssa, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    g1 = (8.0 - ssa * (5.0 + 3.0 * g)) / 4.0
    g2 = 3.0 * ssa * (1.0 - g) / 4.0
    g3 = (2.0 - 3.0 * mu0 * g) / 4.0
    g4 = 1.0 - g3
    return g1, g2, g3, g4


def system_matrix(ssa: float, g: float, mu0: float) -> np.ndarray:
    """A of dy/dtau = A y, y = (U, D, P), for one homogeneous layer."""
    g1, g2, g3, g4 = (float(x) for x in gammas(ssa, g, mu0))
    return np.array([[g1, -g2, -g3 * ssa],
                     [g2, -g1, g4 * ssa],
                     [0.0, 0.0, -1.0 / mu0]])


def column(tau, ssa, g, mu0, albedo, flux_toa=1.0):
    """Fluxes at the nlay+1 levels of a column of homogeneous layers.

    tau, ssa, g: [nlay], layer 0 at the TOA.  flux_toa: solar flux normal
    to the beam at the TOA, so the direct horizontal flux there is
    flux_toa * mu0.  Returns (direct, down_diffuse, up) [nlay+1], in the
    units of flux_toa; level 0 is the TOA, level nlay the surface."""
    tau = np.asarray(tau, dtype=np.float64).reshape(-1)
    ssa = np.asarray(ssa, dtype=np.float64).reshape(-1)
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    nlay = tau.size
    # sub-layers: transfer matrix and count per layer
    trans, counts = [], []
    for l in range(nlay):
        A = system_matrix(ssa[l], g[l], mu0)
        growth = float(np.max(np.abs(np.linalg.eigvals(A[:2, :2]))))
        m = max(1, math.ceil(tau[l] * growth / MAX_GROWTH))
        trans.append(expm(A * (tau[l] / m)))
        counts.append(m)
    nsub = int(sum(counts))
    n = 3 * (nsub + 1)             # unknowns y_0 .. y_nsub, 3 each
    # equations in order: D_0 = 0, P_0 = F; for each sub-layer s the three
    # rows y_{s+1} - E y_s = 0; last U_nsub - albedo (D_nsub + mu0 P_nsub) = 0.
    # Row r of the system has its entries in columns r-2 .. r+3.
    lo, up = 5, 5
    ab = np.zeros((lo + up + 1, n))
    rhs = np.zeros(n)

    def put(row, col, val):
        ab[up + row - col, col] = val

    put(0, 1, 1.0)
    put(1, 2, 1.0)
    rhs[1] = flux_toa
    row, s = 2, 0
    for l in range(nlay):
        E = trans[l]
        for _ in range(counts[l]):
            for i in range(3):
                for j in range(3):
                    put(row + i, 3 * s + j, -E[i, j])
                put(row + i, 3 * (s + 1) + i, 1.0)
            row += 3
            s += 1
    put(row, 3 * nsub, 1.0)
    put(row, 3 * nsub + 1, -albedo)
    put(row, 3 * nsub + 2, -albedo * mu0)
    y = solve_banded((lo, up), ab, rhs).reshape(nsub + 1, 3)
    levels = np.concatenate([[0], np.cumsum(counts)])
    Y = y[levels]
    return mu0 * Y[:, 2], Y[:, 1], Y[:, 0]


def top_of_domain(tau, ssa, g, mu0, albedo, level, flux_toa=1.0):
    """(total downward flux, diffuse fraction) at level `level` of the
    column (the top of the ray tracer's domain)."""
    S, D, _ = column(tau, ssa, g, mu0, albedo, flux_toa)
    tot = S[level] + D[level]
    return tot, (D[level] / tot if tot > 0 else 0.0)
