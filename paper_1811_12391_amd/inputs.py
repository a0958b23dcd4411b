"""Seeded synthetic inputs for the discrete-ordinates CT dose solve.

This module produces the *inputs* of the method and nothing else: the voxel
phantom (material id + density per voxel), the multigroup cross-section
tables, the S_N quadrature set, the source spectrum weights and the source
positions.  It performs none of the transport arithmetic (no ray tracing, no
spherical harmonics, no sweeps, no dose tally), so it can feed both the HIP
library and the FP64 CPU oracle without coupling them.

The paper (Norris & Liu, arXiv:1811.12391) reads its cross sections from the
ORNL 47-group ENDF/B-VII.0 library (Sec. II-D) and its phantoms from CT data
(Sec. II-D); neither is available, so they are replaced by:

* photoelectric mass attenuation K * Z**3.8 * E**-3.2 plus free-electron
  Klein-Nishina Compton scattering, with K calibrated so that water at 20 keV
  has the 13.9 mm mean free path quoted in Sec. II-D;
* group-to-group Compton transfer Legendre moments integrated by Gauss-Legendre
  quadrature over the Klein-Nishina kinematics; photons scattered below the
  lowest group edge are treated as absorbed locally;
* collision-kerma factors (keV cm^2/g) so that dose = sum_g kappa_g * phi_g
  (Sec. II-A: collision kerma taken equal to absorbed dose);
* level-symmetric LQ_N quadrature with N(N+2) directions (Sec. II-A, eq. 3;
  Sec. II-D lists S2..S8 with 8/24/48/80 directions);
* a Kramers 120 kVp photon-number spectrum integrated over each group;
* a water cylinder (Sec. II-D: 35 cm diameter) and a seeded abdomen-like
  phantom built from ellipses.

Conventions used everywhere (shared by the library and the oracle):

* voxel index v = i + nx*(j + ny*k), x fastest; voxel centres at
  origin + (i + 1/2) * dx;
* group g = 0 is the highest energy; edges are listed in descending keV;
* sigma_s[m][l][g_from][g_to] is per unit density (cm^2/g) and nonzero only
  for g_to >= g_from (downscatter only);
* quadrature directions are grouped by octant o = (Ox<0) + 2(Oy<0) + 4(Oz<0),
  weights sum to 4*pi.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CODATA 2018 constants
R_E_CM = 2.8179403262e-13        # classical electron radius, cm
ME_C2_KEV = 510.99895            # electron rest energy, keV
N_A = 6.02214076e23              # Avogadro constant, 1/mol
ZA_WATER = 10.0 / 18.01528       # electrons per nucleon mass unit of water
NE_PER_GRAM = N_A * ZA_WATER     # electrons per gram (same Z/A for every material)

WATER_MFP_20KEV_CM = 1.39        # Sec. II-D: 13.9 mm at 20 keV in water
WATER_MFP_100KEV_CM = 6.06       # Sec. II-D: 60.6 mm at 100 keV in water

# (nominal density g/cm^3, effective Z)
MATERIALS = {
    "air": (1.205e-3, 7.6),
    "water": (1.0, 7.42),
    "soft": (1.04, 7.5),
    "fat": (0.95, 6.3),
    "bone": (1.85, 13.8),
    "lung": (0.26, 7.5),
}


# ----------------------------------------------------------------------------
# Level-symmetric quadrature
# ----------------------------------------------------------------------------

def _lq_points(N: int, mu1: float):
    """Octant points of LQ_N for a given first cosine.

    Returns (cosines mu[0..N/2-1], list of index triples (a,b,c) 0-based with
    a+b+c = N/2 - 1).
    """
    h = N // 2
    if N == 2:
        mu = np.array([1.0 / math.sqrt(3.0)])
    else:
        delta = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (N - 2)
        mu = np.sqrt(mu1 * mu1 + np.arange(h) * delta)
    tri = [(a, b, h - 1 - a - b) for a in range(h) for b in range(h - a)]
    return mu, tri


def _lq_classes(tri):
    classes = {}
    for p, t in enumerate(tri):
        classes.setdefault(tuple(sorted(t)), []).append(p)
    keys = sorted(classes)
    return keys, classes


def _lq_weights(N: int, mu1: float):
    """Point weights (per octant, summing to 1) from the even-moment conditions.

    The number of weight classes c fixes the conditions used: sum w = 1 and
    sum w mu^(2m) = 1/(2m+1) for m = 2..c (the m = 1 condition holds by
    symmetry).  Returns (weights per point, residual of the next condition).
    """
    mu, tri = _lq_points(N, mu1)
    keys, classes = _lq_classes(tri)
    c = len(keys)
    ms = [0] + list(range(2, c + 1))
    A = np.zeros((c, c))
    rhs = np.zeros(c)
    for r, m in enumerate(ms):
        rhs[r] = 1.0 / (2 * m + 1)
        for col, key in enumerate(keys):
            A[r, col] = sum(mu[tri[p][0]] ** (2 * m) for p in classes[key])
    wc = np.linalg.solve(A, rhs)
    w = np.zeros(len(tri))
    for col, key in enumerate(keys):
        for p in classes[key]:
            w[p] = wc[col]
    m_next = c + 1
    resid = sum(w[p] * mu[tri[p][0]] ** (2 * m_next) for p in range(len(tri))) - 1.0 / (2 * m_next + 1)
    return w, resid


def lq_mu1(N: int) -> float:
    """FP64 first cosine of LQ_N: root of the first even-moment condition not
    used to fix the weights (S4: mu^4, S6: mu^6, S8: mu^8)."""
    if N == 2:
        return 1.0 / math.sqrt(3.0)
    from scipy.optimize import brentq

    # mu1 must keep mu_i^2 increasing and below 1: 0 < mu1^2 < 1/3
    f = lambda x: _lq_weights(N, x)[1]
    grid = np.linspace(0.05, math.sqrt(1.0 / 3.0) - 1e-6, 400)
    vals = [f(x) for x in grid]
    for a, b, fa, fb in zip(grid[:-1], grid[1:], vals[:-1], vals[1:]):
        if fa == 0.0:
            return float(a)
        if fa * fb < 0:
            # smallest root with positive weights is the standard LQ_N choice
            r = brentq(f, a, b, xtol=1e-17, rtol=4 * np.finfo(float).eps, maxiter=500)
            w, _ = _lq_weights(N, r)
            if np.all(w > 0):
                return float(r)
    raise ValueError(f"no LQ_{N} first cosine found")


def lq_quadrature(N: int):
    """Level-symmetric S_N set: N(N+2) unit directions and weights summing to 4 pi.

    Directions are ordered by octant o = (Ox<0) + 2(Oy<0) + 4(Oz<0); within an
    octant by the (a, b, c) level triple in lexicographic order.
    """
    if N not in (2, 4, 6, 8):
        raise ValueError("LQ_N supported for N in {2,4,6,8}")
    mu1 = lq_mu1(N)
    mu, tri = _lq_points(N, mu1)
    if N == 2:
        w = np.array([1.0])
    else:
        w, _ = _lq_weights(N, mu1)
    dirs = []
    wts = []
    for o in range(8):
        sx = -1.0 if o & 1 else 1.0
        sy = -1.0 if o & 2 else 1.0
        sz = -1.0 if o & 4 else 1.0
        for p, (a, b, c) in enumerate(tri):
            dirs.append((sx * mu[a], sy * mu[b], sz * mu[c]))
            wts.append(w[p] * (math.pi / 2.0))
    return np.array(dirs, dtype=np.float64), np.array(wts, dtype=np.float64)


# ----------------------------------------------------------------------------
# Synthetic photon cross sections
# ----------------------------------------------------------------------------

def kn_sigma(E_keV):
    """Closed-form Klein-Nishina total cross section per electron (cm^2)."""
    k = np.asarray(E_keV, dtype=np.float64) / ME_C2_KEV
    l = np.log1p(2.0 * k)
    t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k)
    t2 = l / (2.0 * k)
    t3 = (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2
    return 2.0 * math.pi * R_E_CM ** 2 * (t1 + t2 - t3)


def kn_dsigma_domega(E_keV, mu):
    """Klein-Nishina differential cross section per electron (cm^2/sr)."""
    k = np.asarray(E_keV, dtype=np.float64) / ME_C2_KEV
    P = 1.0 / (1.0 + k * (1.0 - mu))
    return 0.5 * R_E_CM ** 2 * P * P * (P + 1.0 / P - (1.0 - mu * mu))


def compton_energy(E_keV, mu):
    return E_keV / (1.0 + (E_keV / ME_C2_KEV) * (1.0 - mu))


def compton_mu(E_keV, Ep_keV):
    """Scattering cosine that takes a photon from E to E'."""
    return 1.0 - ME_C2_KEV * (1.0 / Ep_keV - 1.0 / E_keV)


def photo_constant() -> float:
    """K in mu_pe/rho = K Z^3.8 E^-3.2 (cm^2/g, E in keV), fixed by the water
    mean free path at 20 keV (Sec. II-D)."""
    rho_w, z_w = MATERIALS["water"]
    mu_rho_total = 1.0 / WATER_MFP_20KEV_CM / rho_w
    return (mu_rho_total - NE_PER_GRAM * float(kn_sigma(20.0))) / (z_w ** 3.8 * 20.0 ** -3.2)


def mass_atten(E_keV, Z: float, K: float | None = None):
    """Pointwise mass attenuation (cm^2/g): photoelectric + Klein-Nishina."""
    if K is None:
        K = photo_constant()
    E = np.asarray(E_keV, dtype=np.float64)
    return K * Z ** 3.8 * E ** -3.2 + NE_PER_GRAM * kn_sigma(E)


def group_edges(G: int, e_min: float = 10.0, e_max: float = 120.0):
    """Uniform group edges, descending (g = 0 is the highest energy)."""
    return np.linspace(e_max, e_min, G + 1)


@dataclass
class XSTables:
    edges: np.ndarray          # [G+1] descending keV
    sigma_t: np.ndarray        # [M][G] cm^2/g
    sigma_s: np.ndarray        # [M][L+1][G][G] cm^2/g (from, to)
    kerma: np.ndarray          # [M][G] keV cm^2/g
    cutoff: np.ndarray         # [M][G] cm^2/g scattered below the lowest edge (absorbed)
    names: list = field(default_factory=list)
    Z: np.ndarray = None

    @property
    def G(self):
        return self.sigma_t.shape[1]

    @property
    def M(self):
        return self.sigma_t.shape[0]

    @property
    def L(self):
        return self.sigma_s.shape[1] - 1


def _legendre_table(L: int, mu):
    P = [np.ones_like(mu), mu]
    for l in range(2, L + 1):
        P.append(((2 * l - 1) * mu * P[l - 1] - (l - 1) * P[l - 2]) / l)
    return P[: L + 1]


def compton_transfer(edges, L: int, n_e: int = 64, n_mu: int = 64):
    """Per-electron Compton group transfer Legendre moments (cm^2), the cutoff
    loss (cm^2) and the Compton energy-deposition term (keV cm^2), all as flat
    averages over the source group.

    Returns (T[L+1][G][G], cut[G], edep[G], sig_kn[G]).
    """
    G = len(edges) - 1
    e_min = edges[-1]
    xe, we = np.polynomial.legendre.leggauss(n_e)
    xm, wm = np.polynomial.legendre.leggauss(n_mu)
    T = np.zeros((L + 1, G, G))
    cut = np.zeros(G)
    edep = np.zeros(G)
    sig = np.zeros(G)
    for gf in range(G):
        ehi, elo = edges[gf], edges[gf + 1]
        E = 0.5 * (ehi + elo) + 0.5 * (ehi - elo) * xe       # nodes in the source group
        wE = 0.5 * we                                          # flat average weights (sum 1)
        sig[gf] = np.sum(wE * kn_sigma(E))
        for iE, (Ei, wi) in enumerate(zip(E, wE)):
            # energy deposited by Compton: integral of (E - E') dsigma over all angles
            mu = xm
            dmu = np.ones_like(mu)
            ds = kn_dsigma_domega(Ei, mu) * 2.0 * math.pi
            edep[gf] += wi * np.sum(wm * ds * (Ei - compton_energy(Ei, mu)) * dmu)
            ep_min = Ei / (1.0 + 2.0 * Ei / ME_C2_KEV)
            for gt in range(gf, G):
                lo = max(edges[gt + 1], ep_min)
                hi = min(edges[gt], Ei)
                if hi <= lo:
                    continue
                a, b = compton_mu(Ei, lo), compton_mu(Ei, hi)
                a, b = max(a, -1.0), min(b, 1.0)
                if b <= a:
                    continue
                m = 0.5 * (a + b) + 0.5 * (b - a) * xm
                wmu = 0.5 * (b - a) * wm
                ds = kn_dsigma_domega(Ei, m) * 2.0 * math.pi
                P = _legendre_table(L, m)
                for l in range(L + 1):
                    T[l, gf, gt] += wi * np.sum(wmu * ds * P[l])
            if ep_min < e_min:
                a, b = -1.0, min(compton_mu(Ei, e_min), 1.0)
                if b > a:
                    m = 0.5 * (a + b) + 0.5 * (b - a) * xm
                    wmu = 0.5 * (b - a) * wm
                    ds = kn_dsigma_domega(Ei, m) * 2.0 * math.pi
                    cut[gf] += wi * np.sum(wmu * ds)
                    # energy of the photons below the cutoff is deposited too
                    edep[gf] += wi * np.sum(wmu * ds * compton_energy(Ei, m))
    return T, cut, edep, sig


def xs_tables(material_names, G: int, L: int, e_min: float = 10.0, e_max: float = 120.0) -> XSTables:
    """Multigroup tables per unit density for the named materials."""
    edges = group_edges(G, e_min, e_max)
    K = photo_constant()
    T, cut, edep, sig_kn = compton_transfer(edges, L)
    M = len(material_names)
    st = np.zeros((M, G))
    ss = np.zeros((M, L + 1, G, G))
    ka = np.zeros((M, G))
    cu = np.zeros((M, G))
    Zs = np.zeros(M)
    for m, name in enumerate(material_names):
        _, Z = MATERIALS[name]
        Zs[m] = Z
        for g in range(G):
            ehi, elo = edges[g], edges[g + 1]
            dE = ehi - elo
            pe = K * Z ** 3.8 * (ehi ** -2.2 - elo ** -2.2) / (-2.2 * dE)
            epe = K * Z ** 3.8 * (ehi ** -1.2 - elo ** -1.2) / (-1.2 * dE)
            st[m, g] = pe + NE_PER_GRAM * sig_kn[g]
            ka[m, g] = epe + NE_PER_GRAM * edep[g]
            cu[m, g] = NE_PER_GRAM * cut[g]
        ss[m] = NE_PER_GRAM * T
    return XSTables(edges=edges, sigma_t=st, sigma_s=ss, kerma=ka, cutoff=cu,
                    names=list(material_names), Z=Zs)


def kramers_weights(edges, E0: float = 120.0):
    """Group photon weights of a Kramers spectrum dN/dE ~ (E0 - E)/E, normalised
    to sum 1; ordered like the groups (g = 0 highest energy)."""
    edges = np.asarray(edges, dtype=np.float64)
    hi, lo = edges[:-1], edges[1:]
    w = E0 * np.log(hi / lo) - (hi - lo)
    return w / w.sum()


# ----------------------------------------------------------------------------
# Phantoms and sources
# ----------------------------------------------------------------------------

@dataclass
class Phantom:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    origin: np.ndarray         # [3] corner of the grid (cm)
    material: np.ndarray       # [C] uint8
    density: np.ndarray        # [C] float64
    material_names: list

    @property
    def C(self):
        return self.nx * self.ny * self.nz

    def centres(self):
        x = self.origin[0] + (np.arange(self.nx) + 0.5) * self.dx
        y = self.origin[1] + (np.arange(self.ny) + 0.5) * self.dy
        z = self.origin[2] + (np.arange(self.nz) + 0.5) * self.dz
        return x, y, z


def _centred_origin(nx, ny, nz, dx, dy, dz):
    return np.array([-nx * dx / 2.0, -ny * dy / 2.0, -nz * dz / 2.0])


def cylinder_phantom(nx, ny, nz, d, radius=17.5, names=("air", "water")) -> Phantom:
    """Water cylinder along z (all of z) in air; classification by voxel centre."""
    origin = _centred_origin(nx, ny, nz, d, d, d)
    x = origin[0] + (np.arange(nx) + 0.5) * d
    y = origin[1] + (np.arange(ny) + 0.5) * d
    X, Y = np.meshgrid(x, y, indexing="xy")          # [ny][nx]
    inside = (X * X + Y * Y) <= radius * radius
    mat2 = np.where(inside, 1, 0).astype(np.uint8)
    mat = np.broadcast_to(mat2, (nz, ny, nx)).reshape(-1).copy()
    dens_tab = np.array([MATERIALS[n][0] for n in names])
    dens = dens_tab[mat].astype(np.float64)
    return Phantom(nx, ny, nz, d, d, d, origin, mat, dens, list(names))


ABDOMEN_NAMES = ("air", "fat", "soft", "lung", "bone")


def abdomen_phantom(nx, ny, nz, d, seed: int = 1811) -> Phantom:
    """Seeded abdomen-like phantom from ellipses (painted in order, later
    painters override earlier ones), plus 2% Gaussian density noise on non-air
    voxels.  Random draws, in order, from numpy.random.default_rng(seed): for
    each ellipse a centre jitter U(-0.5, 0.5) cm per axis and a semi-axis
    scale U(0.95, 1.05) per axis (ribs first draw their angle jitter
    U(-10, 10) degrees); then one N(0,1) per voxel in index order (air voxels
    draw too, their density is left nominal)."""
    rng = np.random.default_rng(seed)
    origin = _centred_origin(nx, ny, nz, d, d, d)
    x = origin[0] + (np.arange(nx) + 0.5) * d
    y = origin[1] + (np.arange(ny) + 0.5) * d
    z = origin[2] + (np.arange(nz) + 0.5) * d
    X, Y = np.meshgrid(x, y, indexing="xy")
    idx = {n: i for i, n in enumerate(ABDOMEN_NAMES)}
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)

    def ellipse(cx, cy, ax, ay):
        jx, jy = rng.uniform(-0.5, 0.5, size=2)
        sx, sy = rng.uniform(0.95, 1.05, size=2)
        cx, cy, ax, ay = cx + jx, cy + jy, ax * sx, ay * sy
        return ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 <= 1.0

    body = ellipse(0.0, 0.0, 16.5, 12.0)
    mat[:, body] = idx["fat"]
    inner = ellipse(0.0, 0.0, 15.0, 10.5)
    mat[:, inner] = idx["soft"]
    upper = z > 0.0
    for sgn in (1.0, -1.0):
        lung = ellipse(sgn * 7.5, 3.5, 4.0, 3.0)
        for k in np.nonzero(upper)[0]:
            mat[k, lung] = idx["lung"]
    vert = ellipse(0.0, -7.5, 2.0, 1.8)
    mat[:, vert] = idx["bone"]
    spin = ellipse(0.0, -10.0, 0.8, 1.5)
    mat[:, spin] = idx["bone"]
    for ang in (30, 60, 120, 150, 210, 240, 300, 330):
        a = math.radians(ang + rng.uniform(-10.0, 10.0))
        rib = ellipse(13.8 * math.cos(a), 9.5 * math.sin(a), 0.6, 0.4)
        mat[:, rib] = idx["bone"]
    mat = mat.reshape(-1)
    noise = rng.standard_normal(mat.size)
    dens_tab = np.array([MATERIALS[n][0] for n in ABDOMEN_NAMES])
    dens = dens_tab[mat] * np.where(mat != idx["air"], 1.0 + 0.02 * noise, 1.0)
    return Phantom(nx, ny, nz, d, d, d, origin, mat, dens.astype(np.float64), list(ABDOMEN_NAMES))


def top_source(distance=54.0):
    """Single point source on the +y side aimed at the z axis (toward -y)."""
    return np.array([[0.0, distance, 0.0]]), np.array([[0.0, -1.0, 0.0]])


def ring_sources(n=36, step_deg=10.0, distance=54.0):
    """Axial-scan positions on a circle in the z = 0 plane, each aimed at the
    z axis: p_k = d (sin(k step), cos(k step), 0)."""
    a = np.radians(step_deg * np.arange(n))
    pos = np.stack([distance * np.sin(a), distance * np.cos(a), np.zeros(n)], axis=1)
    axis = -pos / np.linalg.norm(pos, axis=1, keepdims=True)
    return pos, axis


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    phantom: Phantom
    xs: XSTables
    dirs: np.ndarray
    weights: np.ndarray
    L: int
    src_pos: np.ndarray
    src_axis: np.ndarray
    fan_deg: float
    cone_deg: float
    group_w: np.ndarray
    tol: float = 1e-6
    max_iter: int = 1000
    precision: str = "fp64"
    extra: dict = field(default_factory=dict)

    @property
    def G(self):
        return self.xs.G

    @property
    def N(self):
        return self.dirs.shape[0]

    @property
    def B(self):
        return self.src_pos.shape[0]


def make_problem(name: str) -> Problem:
    """The five workloads (water cylinder and abdomen phantoms) plus small
    ragged test cases.  'c1'..'c5' follow the configurations used for the
    measurements; 'ct16' is the superposed CT-scan form; 'tiny*' are
    few-second oracle sizes."""
    fan, cone = 20.0, 10.0          # beam window (full angles, degrees)
    if name == "c1":
        ph = cylinder_phantom(24, 24, 8, 1.5)
        G, S, L, pos, axis, prec = 4, 4, 1, *top_source(), "fp64"
    elif name == "c2":
        ph = cylinder_phantom(64, 64, 16, 0.6)
        G, S, L, pos, axis, prec = 19, 8, 3, *top_source(), "fp64"
    elif name == "c3":
        ph = abdomen_phantom(128, 128, 32, 0.3)
        G, S, L, pos, axis, prec = 19, 8, 3, *top_source(), "fp32"
    elif name == "c4":
        ph = cylinder_phantom(64, 64, 16, 0.6)
        G, S, L, (pos, axis), prec = 19, 6, 3, ring_sources(), "fp32"
    elif name == "c5":
        ph = abdomen_phantom(64, 64, 16, 0.6)
        G, S, L, pos, axis, prec = 19, 6, 3, *top_source(), "fp32"
    elif name == "ct16":
        # CT-scan form: 16 cone beams of 30 degrees evenly on the 54 cm circle
        # around the c2 cylinder, meant to be superposed into one collided solve
        ph = cylinder_phantom(64, 64, 16, 0.6)
        G, S, L, (pos, axis), prec = 19, 6, 3, ring_sources(16, 22.5), "fp32"
        fan = cone = 30.0
    elif name == "tiny_ct":
        ph = cylinder_phantom(13, 11, 5, 3.0)
        G, S, L, (pos, axis), prec = 3, 4, 1, ring_sources(4, 90.0), "fp64"
        fan = cone = 30.0
    elif name == "tiny":
        # ragged: not a multiple of any tile, several groups, P1
        ph = cylinder_phantom(13, 11, 5, 3.0)
        G, S, L, pos, axis, prec = 3, 4, 1, *top_source(), "fp64"
    elif name == "tiny_abd":
        ph = abdomen_phantom(21, 19, 6, 1.8)
        G, S, L, pos, axis, prec = 5, 6, 3, *top_source(), "fp64"
    else:
        raise ValueError(name)
    xs = xs_tables(ph.material_names, G, L)
    dirs, w = lq_quadrature(S)
    gw = kramers_weights(xs.edges)
    return Problem(name, ph, xs, dirs, w, L, pos, axis, fan, cone, gw, precision=prec)
