"""Independent reference solutions that pin the oracle (and through it the
GPU path) to the physics the paper states (sec. 2.3), not to itself.

  * Beer-Lambert direct beam through horizontally uniform layers.
  * Non-scattering absorbing layers over a Lambertian surface: the reflected
    radiance is isotropic, so the escape probability through optical depth
    t is 2 E_3(t) and each layer's share follows from differences of E_3.
  * Isotropically scattering plane-parallel slab (any vertical extinction
    profile, uniform omega) with collimated incidence and a Lambertian
    surface: the collision density obeys the Schwarzschild-Milne integral
    equation  f(t) = exp(-t/mu0)/mu0 + a S 2E_2(tau1 - t)
                   + omega * int 1/2 E_1(|t - t'|) f(t') dt'
    (Chandrasekhar 1950), solved by a piecewise-constant Galerkin method with
    exactly integrated cell kernels (differences of E_3).
  * An analog Monte Carlo on tiny grids: regular (cell-by-cell) tracking, no
    weights, no majorants, absorption and surface absorption by sampling,
    phase functions and the Lambertian law sampled by rejection.  It shares
    no step with the weighted null-collision algorithm beyond the physics.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expn


def E(n, x):
    x = np.asarray(x, dtype=np.float64)
    out = np.where(x == 0.0, 1.0 / (n - 1) if n > 1 else np.inf, 0.0)
    pos = x > 0.0
    out = np.array(out, dtype=np.float64)
    out[pos] = expn(n, x[pos])
    return out


def sun_direction(sza_deg, az_deg):
    th, ph = np.radians(sza_deg), np.radians(az_deg)
    return np.array([-np.sin(th) * np.sin(ph), -np.sin(th) * np.cos(ph), -np.cos(th)])


# ---------------------------------------------------------------------------
# Beer-Lambert and the absorbing slab over a Lambertian surface
# ---------------------------------------------------------------------------

def beer_lambert(tau_col, mu0):
    return np.exp(-np.asarray(tau_col) / mu0)


def absorbing_layers_lambertian(dtau_layers, mu0, albedo):
    """Pure absorber (omega = 0) with layer optical depths dtau_layers
    (index 0 = bottom layer), collimated incidence mu0, Lambertian albedo.

    Returns dict of per-photon expectations: sfc_dir, sfc_abs, toa_up,
    abs_dir[k], abs_dif[k]."""
    dt = np.asarray(dtau_layers, dtype=np.float64)
    nz = dt.size
    tau_top = np.concatenate([np.cumsum(dt[::-1])[::-1][1:], [0.0]])  # optical depth above each layer
    tau_bot = np.concatenate([[0.0], np.cumsum(dt)[:-1]])            # optical depth below each layer
    tau1 = dt.sum()
    T = np.exp(-tau1 / mu0)
    abs_dir = np.exp(-tau_top / mu0) * (1.0 - np.exp(-dt / mu0))
    up = albedo * T
    abs_dif = up * 2.0 * (E(3, tau_bot) - E(3, tau_bot + dt))
    return {
        "sfc_dir": T,
        "sfc_dif": 0.0,
        "sfc_abs": (1.0 - albedo) * T,
        "toa_up": up * 2.0 * E(3, tau1),
        "abs_dir": abs_dir,
        "abs_dif": abs_dif,
    }


def direct_heating_uniform_layers(k_ext_z, k_abs_z, dz, mu0):
    """Expected direct-beam absorption per layer (index 0 = bottom):
    exp(-tau_above/mu0) (k_abs/k_ext) (1 - exp(-k_ext dz / mu0))."""
    ke = np.asarray(k_ext_z, dtype=np.float64)
    ka = np.asarray(k_abs_z, dtype=np.float64)
    dt = ke * dz
    tau_top = np.concatenate([np.cumsum(dt[::-1])[::-1][1:], [0.0]])
    frac = np.where(ke > 0, ka / np.where(ke > 0, ke, 1.0), 0.0)
    return np.exp(-tau_top / mu0) * frac * (1.0 - np.exp(-dt / mu0))


# ---------------------------------------------------------------------------
# Isotropic slab: Milne integral equation, Galerkin with exact cell kernels
# ---------------------------------------------------------------------------

def isotropic_slab(dtau_layers, omega, mu0, albedo=0.0, cells_per_unit=400, min_cells=8):
    """Plane-parallel slab (layer optical depths dtau_layers, index 0 =
    bottom), uniform single-scattering albedo omega, isotropic phase
    function, collimated incidence with cosine mu0 at the top, Lambertian
    surface of the given albedo.  Returns per-photon expectations."""
    dt = np.asarray(dtau_layers, dtype=np.float64)
    dt_top_first = dt[::-1]                      # optical depth measured from the top
    edges_layers = np.concatenate([[0.0], np.cumsum(dt_top_first)])
    tau1 = edges_layers[-1]
    # sub-cells of each layer (uniform within a layer)
    sub_edges = [0.0]
    owner = []
    for L in range(dt_top_first.size):
        n = max(min_cells, int(np.ceil(dt_top_first[L] * cells_per_unit))) if dt_top_first[L] > 0 else 0
        for c in range(n):
            sub_edges.append(edges_layers[L] + (c + 1) * dt_top_first[L] / n)
            owner.append(L)
    a = np.array(sub_edges[:-1])
    b = np.array(sub_edges[1:])
    h = b - a
    M = a.size
    owner = np.array(owner)

    # K[i, j] = (1/h_i) int_i int_j 1/2 E1(|t - t'|) dt' dt
    ai, bi = a[:, None], b[:, None]
    aj, bj = a[None, :], b[None, :]

    # For intervals I=[ai,bi], J=[aj,bj]:
    # int_I int_J 1/2 E1(|t-t'|) = G(bi-aj) - G(ai-aj) - G(bi-bj) + G(ai-bj)
    # with G'' = 1/2 E1(|x|) and G' continuous at 0: G(x) = |x|/2 + E3(|x|)/2
    def G(x):
        x = np.abs(x)
        return 0.5 * x + 0.5 * E(3, x)

    Kint = G(bi - aj) - G(ai - aj) - G(bi - bj) + G(ai - bj)
    K = Kint / h[:, None]
    f0 = (np.exp(-a / mu0) - np.exp(-b / mu0)) / h            # cell average of exp(-t/mu0)/mu0
    gL = 2.0 * (E(3, tau1 - b) - E(3, tau1 - a)) / h            # cell average of 2 E2(tau1 - t)
    down = 0.5 * (E(3, tau1 - b) - E(3, tau1 - a))              # int_i 1/2 E2(tau1 - t) dt
    up = 0.5 * (E(3, a) - E(3, b))                               # int_i 1/2 E2(t) dt
    T = np.exp(-tau1 / mu0)
    # unknowns x = [f_1..f_M, S]
    A = np.zeros((M + 1, M + 1))
    A[:M, :M] = np.eye(M) - omega * K
    A[:M, M] = -albedo * gL
    A[M, :M] = -omega * down
    A[M, M] = 1.0
    rhs = np.concatenate([f0, [T]])
    x = np.linalg.solve(A, rhs)
    f, S = x[:M], x[M]
    R = omega * np.sum(f * up) + albedo * S * 2.0 * E(3, tau1)
    coll = f * h
    nl = dt_top_first.size
    abs_layer = np.bincount(owner, weights=(1.0 - omega) * coll, minlength=nl)
    abs_dir_layer = np.bincount(owner, weights=(1.0 - omega) * f0 * h, minlength=nl)
    return {
        "toa_up": R,
        "sfc_dir": T,
        "sfc_dif": S - T,
        "sfc_abs": (1.0 - albedo) * S,
        "abs_dir": abs_dir_layer[::-1],          # back to index 0 = bottom
        "abs_dif": (abs_layer - abs_dir_layer)[::-1],
    }


# ---------------------------------------------------------------------------
# Analog Monte Carlo on tiny grids (vectorised over photons)
# ---------------------------------------------------------------------------

def _rejection(rng, n, pdf, pmax):
    out = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        mu = rng.uniform(-1.0, 1.0, todo.size)
        acc = rng.uniform(0.0, pmax, todo.size) < pdf(mu)
        out[todo[acc]] = mu[acc]
        todo = todo[~acc]
    return out


def _hg_pdf(g):
    return lambda mu: 0.5 * (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5


def _rotate(d, mu, phi):
    """Rodrigues-style rotation: tilt d by acos(mu) about an axis
    perpendicular to d, then spin by phi about d."""
    n = d.shape[0]
    ref = np.where(np.abs(d[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    ax = np.cross(d, ref)
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    st = np.sqrt(np.maximum(0.0, 1 - mu * mu))[:, None]
    # vector at angle theta from d in the plane of d and ax x d, then spin
    perp = np.cross(ax, d)
    v = mu[:, None] * d + st * perp
    # rotate v about d by phi (Rodrigues)
    c, s = np.cos(phi)[:, None], np.sin(phi)[:, None]
    v = v * c + np.cross(d, v) * s + d * np.sum(d * v, axis=1, keepdims=True) * (1 - c)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def analog_mc(fields, sza, azimuth, n_photons, rng, diffuse_fraction=0.0, max_events=100000):
    """Analog MC of the same radiative-transfer problem.  Returns per-photon
    tally densities: arrays of counts divided by photons per column."""
    grid = fields.grid
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    dx, dy, dz = grid.dx, grid.dy, grid.dz
    Lx, Ly, H = nx * dx, ny * dy, nz * dz
    ke = fields.k_ext.astype(np.float64)
    kc = fields.k_ext_cloud.astype(np.float64)
    om = fields.ssa.astype(np.float64)
    gg = fields.g.astype(np.float64)
    alb = fields.albedo.astype(np.float64)

    out = {k: np.zeros(grid.shape3) for k in ("abs_dir", "abs_dif")}
    out.update({k: np.zeros(grid.shape2) for k in ("sfc_dir", "sfc_dif", "sfc_abs", "toa_up")})

    # emission: uniform over the top (equivalent in law to systematic sampling)
    x = rng.uniform(0, Lx, n_photons)
    y = rng.uniform(0, Ly, n_photons)
    z = np.full(n_photons, H)
    d = np.tile(sun_direction(sza, azimuth), (n_photons, 1))
    direct = np.ones(n_photons, dtype=bool)
    diff = rng.uniform(size=n_photons) < diffuse_fraction
    if diff.any():
        m = diff.sum()
        mu = _rejection(rng, m, lambda u: np.where(u > 0, u, 0.0), 1.0)  # pdf prop. to mu on (0,1)
        ph = rng.uniform(0, 2 * np.pi, m)
        st = np.sqrt(1 - mu * mu)
        d[diff] = np.stack([st * np.cos(ph), st * np.sin(ph), -mu], axis=1)
        direct[diff] = False
    i = np.minimum((x / dx).astype(np.int64), nx - 1)
    j = np.minimum((y / dy).astype(np.int64), ny - 1)
    k = np.full(n_photons, nz - 1)
    alive = np.arange(n_photons)
    tau = rng.exponential(size=n_photons)
    for _ in range(max_events):
        if alive.size == 0:
            break
        a = alive
        dd = d[a]
        with np.errstate(divide="ignore", invalid="ignore"):
            tx = np.where(dd[:, 0] > 0, ((i[a] + 1) * dx - x[a]) / dd[:, 0],
                          np.where(dd[:, 0] < 0, (i[a] * dx - x[a]) / dd[:, 0], np.inf))
            ty = np.where(dd[:, 1] > 0, ((j[a] + 1) * dy - y[a]) / dd[:, 1],
                          np.where(dd[:, 1] < 0, (j[a] * dy - y[a]) / dd[:, 1], np.inf))
            tz = np.where(dd[:, 2] > 0, ((k[a] + 1) * dz - z[a]) / dd[:, 2],
                          np.where(dd[:, 2] < 0, (k[a] * dz - z[a]) / dd[:, 2], np.inf))
        tx, ty, tz = np.maximum(tx, 0), np.maximum(ty, 0), np.maximum(tz, 0)
        t_exit = np.minimum(np.minimum(tx, ty), tz)
        kk = ke[k[a], j[a], i[a]]
        s_coll = np.where(kk > 0, tau[a] / np.where(kk > 0, kk, 1.0), np.inf)
        coll = s_coll < t_exit
        # --- photons that collide inside their cell
        ac = a[coll]
        if ac.size:
            s = s_coll[coll][:, None]
            x[ac] += s[:, 0] * d[ac, 0]
            y[ac] += s[:, 0] * d[ac, 1]
            z[ac] += s[:, 0] * d[ac, 2]
            ci, cj, ck = i[ac], j[ac], k[ac]
            u = rng.uniform(size=ac.size)
            absorbed = u >= om[ck, cj, ci]
            ab = ac[absorbed]
            np.add.at(out["abs_dir"], (k[ab][direct[ab]], j[ab][direct[ab]], i[ab][direct[ab]]), 1.0)
            nd = ~direct[ab]
            np.add.at(out["abs_dif"], (k[ab][nd], j[ab][nd], i[ab][nd]), 1.0)
            sc = ac[~absorbed]
            if sc.size:
                u2 = rng.uniform(size=sc.size)
                cloud = u2 * ke[k[sc], j[sc], i[sc]] < kc[k[sc], j[sc], i[sc]]
                mu = np.empty(sc.size)
                # Rayleigh by rejection: pdf 3/8 (1 + mu^2), max 3/4
                nr = (~cloud).sum()
                if nr:
                    mu[~cloud] = _rejection(rng, nr, lambda m: 0.375 * (1 + m * m), 0.75)
                if cloud.any():
                    gvals = gg[k[sc][cloud], j[sc][cloud], i[sc][cloud]]
                    mu_c = np.empty(gvals.size)
                    for gv in np.unique(gvals):
                        sel = gvals == gv
                        pmax = _hg_pdf(gv)(np.sign(gv) if gv != 0 else 1.0)
                        mu_c[sel] = _rejection(rng, sel.sum(), _hg_pdf(gv), pmax)
                    mu[cloud] = mu_c
                phi = rng.uniform(0, 2 * np.pi, sc.size)
                d[sc] = _rotate(d[sc], mu, phi)
                direct[sc] = False
            tau[sc] = rng.exponential(size=sc.size)
            alive = np.setdiff1d(alive, ab, assume_unique=True)
        # --- photons that reach their cell boundary
        ab_ = a[~coll]
        if ab_.size:
            te = t_exit[~coll]
            tau[ab_] -= kk[~coll] * te
            x[ab_] += te * d[ab_, 0]
            y[ab_] += te * d[ab_, 1]
            z[ab_] += te * d[ab_, 2]
            txa, tya, tza = tx[~coll], ty[~coll], tz[~coll]
            ax_z = tza <= np.minimum(txa, tya)
            ax_x = (~ax_z) & (txa <= tya)
            ax_y = (~ax_z) & (~ax_x)
            # x crossings
            px = ab_[ax_x]
            up = d[px, 0] > 0
            i[px] = np.where(up, i[px] + 1, i[px] - 1)
            wrap_hi = i[px] == nx
            wrap_lo = i[px] < 0
            i[px] = np.where(wrap_hi, 0, np.where(wrap_lo, nx - 1, i[px]))
            x[px] = np.where(up, i[px] * dx, (i[px] + 1) * dx)
            py = ab_[ax_y]
            up = d[py, 1] > 0
            j[py] = np.where(up, j[py] + 1, j[py] - 1)
            wrap_hi = j[py] == ny
            wrap_lo = j[py] < 0
            j[py] = np.where(wrap_hi, 0, np.where(wrap_lo, ny - 1, j[py]))
            y[py] = np.where(up, j[py] * dy, (j[py] + 1) * dy)
            pz = ab_[ax_z]
            up = d[pz, 2] > 0
            esc = pz[up & (k[pz] == nz - 1)]
            sfc = pz[(~up) & (k[pz] == 0)]
            mid = pz[~((up & (k[pz] == nz - 1)) | ((~up) & (k[pz] == 0)))]
            upm = d[mid, 2] > 0
            k[mid] = np.where(upm, k[mid] + 1, k[mid] - 1)
            z[mid] = np.where(upm, k[mid] * dz, (k[mid] + 1) * dz)
            np.add.at(out["toa_up"], (j[esc], i[esc]), 1.0)
            if sfc.size:
                dr = direct[sfc]
                np.add.at(out["sfc_dir"], (j[sfc][dr], i[sfc][dr]), 1.0)
                np.add.at(out["sfc_dif"], (j[sfc][~dr], i[sfc][~dr]), 1.0)
                absorb = rng.uniform(size=sfc.size) >= alb[j[sfc], i[sfc]]
                sa = sfc[absorb]
                np.add.at(out["sfc_abs"], (j[sa], i[sa]), 1.0)
                rf = sfc[~absorb]
                mu = _rejection(rng, rf.size, lambda u: np.where(u > 0, u, 0.0), 1.0)
                ph = rng.uniform(0, 2 * np.pi, rf.size)
                st = np.sqrt(1 - mu * mu)
                d[rf] = np.stack([st * np.cos(ph), st * np.sin(ph), mu], axis=1)
                direct[rf] = False
                z[rf] = 0.0
                tau[rf] = rng.exponential(size=rf.size)
                alive = np.setdiff1d(alive, sa, assume_unique=True)
            alive = np.setdiff1d(alive, esc, assume_unique=True)
    per_col = n_photons / grid.ncol
    return {k_: v / per_col for k_, v in out.items()}
