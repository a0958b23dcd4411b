"""Pins of the oracle's anisotropic scattering source (eq. 2 with the
scattering kernel expanded in Legendre polynomials, Sec. II-A) and of its dose
tally, against things other than the oracle itself:

- the direction-to-direction form of eq. (2): the source a direction n gets
  from the angular flux of every direction n' is
  sum_n' w_n' sum_l (2l+1)/(4 pi) rho s_l P_l(Omega_n . Omega_n') psi_n'
  (Legendre polynomials from numpy), for the within-group and the downscatter
  transfer, S4-S8 at P1-P3;
- the anisotropic infinite homogeneous medium: a uniform source with moments
  S_g,lm and the matching angular inflow give the closed form
  phi_g,lm = (S_g,lm + sum_{g'<g} rho s_l^{g'g} phi_g',lm) / (rho (t_g - s_l^{gg}));
- energy conservation of the dose tally for a pure absorber whose kerma factor
  is the group energy times its attenuation coefficient.

The first two fail if any moment of degree l >= 1 scatters with the wrong
Legendre coefficient (s_0 in place of s_l, say), in either group term."""
import math

import numpy as np
import pytest

from paper_1811_12391_amd import inputs as I


def _legendre(l, x):
    return np.polynomial.legendre.legval(x, [0] * l + [1])


def _random_tables(rng, M, L, G):
    """Random transfer moments s_l^{g->g'} (from, to): zero for g' < g
    (downscatter only), positive and different in every degree l."""
    ss = np.zeros((M, L + 1, G, G))
    for gf in range(G):
        for gt in range(gf, G):
            ss[:, :, gf, gt] = rng.uniform(0.2, 1.0, (M, L + 1))
    return ss


@pytest.mark.parametrize("N,L", [(4, 1), (4, 2), (6, 1), (6, 2), (6, 3), (8, 1), (8, 2), (8, 3)])
def test_scatter_source_direction_form(oracle_mod, N, L):
    """moments -> scatter moments -> directions equals the direction-to-
    direction sum of eq. (2) for a random anisotropic angular flux, within the
    group and for downscatter."""
    rng = np.random.default_rng(100 + 10 * N + L)
    d, w = I.lq_quadrature(N)
    Nd, C, M, G = d.shape[0], 7, 3, 3
    mat = rng.integers(0, M, C).astype(np.uint8)
    rho = rng.uniform(0.3, 2.0, C)
    ss = _random_tables(rng, M, L, G)
    psi = rng.uniform(-0.5, 1.5, (Nd, C))
    Mm, Dm = oracle_mod.moment_maps(L, d, w)
    phi = Dm @ psi                                        # [Nm][C]
    cosines = d @ d.T                                     # [N][N']
    for gf, gt in [(0, 0), (1, 1), (0, 1), (0, 2), (1, 2)]:
        S = oracle_mod.scatter_moments(mat, rho, ss, L, gf, gt, phi)
        q = Mm @ S                                        # [N][C]
        ref = np.zeros((Nd, C))
        for l in range(L + 1):
            kern = (2 * l + 1) / (4 * math.pi) * _legendre(l, cosines) * w[None, :]   # [N][N']
            ref += (kern @ psi) * (rho * ss[mat, l, gf, gt])[None, :]
        assert np.allclose(q, ref, rtol=0, atol=1e-13 * np.abs(ref).max()), (gf, gt)


def test_scatter_source_accumulates_on_base(oracle_mod):
    """out = base + rho s_l phi, element by element."""
    rng = np.random.default_rng(7)
    L, C, M, G = 2, 5, 2, 2
    mat = rng.integers(0, M, C).astype(np.uint8)
    rho = rng.uniform(0.5, 1.5, C)
    ss = _random_tables(rng, M, L, G)
    phi = rng.standard_normal(((L + 1) ** 2, C))
    base = rng.standard_normal(((L + 1) ** 2, C))
    lof = np.array([l for l in range(L + 1) for _ in range(2 * l + 1)])
    out = oracle_mod.scatter_moments(mat, rho, ss, L, 0, 1, phi, base=base)
    ref = base + rho[None, :] * ss[mat][:, lof, 0, 1].T * phi
    assert np.allclose(out, ref, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("N,L", [(6, 3), (8, 3), (8, 2)])
def test_infinite_medium_anisotropic(oracle_mod, N, L):
    """A uniform anisotropic source in an infinite homogeneous medium (the
    boundary inflow in every direction is the infinite-medium angular flux)
    gives every flux moment in closed form, group by group."""
    rng = np.random.default_rng(200 + N + L)
    G = 4
    ph = I.cylinder_phantom(5, 4, 3, 1.0)
    ph.material[:] = 1
    rho = 1.3
    ph.density[:] = rho
    xs = I.xs_tables(ph.material_names, G, L)
    st, ss = xs.sigma_t[1], xs.sigma_s[1]              # [G], [L+1][G][G]
    Nm = (L + 1) ** 2
    lof = np.array([l for l in range(L + 1) for _ in range(2 * l + 1)])
    S = np.zeros((G, Nm))
    S[:, 0] = rng.uniform(0.5, 2.0, G)
    S[:, 1:] = rng.uniform(-0.04, 0.04, (G, Nm - 1)) * S[:, :1]
    phi = np.zeros((G, Nm))
    for g in range(G):
        num = S[g] + sum(rho * ss[lof, gp, g] * phi[gp] for gp in range(g))
        phi[g] = num / (rho * (st[g] - ss[lof, g, g]))
    # the scatter moments of degree >= 1 differ from s_0, so they matter here
    assert np.all(np.abs(ss[1:, np.arange(G), np.arange(G)] - ss[0, np.arange(G), np.arange(G)]) > 0.01 * st)
    d, w = I.lq_quadrature(N)
    Mm, _ = oracle_mod.moment_maps(L, d, w)
    inflow = phi @ Mm.T                                  # [G][N] angular flux of the infinite medium
    assert inflow.min() > 0                              # no set-to-zero fixup is involved
    ext = np.repeat(S[:, :, None], ph.C, axis=2)
    out, dose, iters, eps, bal = oracle_mod.solve_fixed(ph, xs, d, w, L, ext, inflow, tol=1e-14)
    for g in range(G):
        assert np.allclose(out[g], phi[g][:, None], rtol=0, atol=1e-11 * phi[g, 0]), g
    # the balance closes with the anisotropic source: P = R + L
    P, R, Lk = bal.T
    assert np.all(np.abs(P - R - Lk) <= 1e-10 * P)


def test_dose_energy_conservation_pure_absorber(oracle_mod):
    """Pure absorber (no scattering) whose kerma factor is the group's energy
    times its mass attenuation coefficient: every photon deposits its energy
    where it is absorbed, so in an infinite medium the deposited energy per
    volume, rho * dose, equals the emitted energy per volume sum_g E_g S_g."""
    G, L = 3, 0
    ph = I.cylinder_phantom(4, 4, 3, 0.8)
    ph.material[:] = 1
    rho = 1.7
    ph.density[:] = rho
    xs = I.xs_tables(ph.material_names, G, L)
    xs.sigma_s[:] = 0.0
    E = 0.5 * (xs.edges[:-1] + xs.edges[1:])                 # keV per photon of group g
    xs.kerma[:] = E[None, :] * xs.sigma_t
    S = np.array([0.7, 1.9, 0.4])                             # photons / cm^3 per source photon
    phi = S / (rho * xs.sigma_t[1])
    d, w = I.lq_quadrature(4)
    ext = np.repeat(S[:, None, None], ph.C, axis=2)
    inflow = np.repeat((phi / (4 * math.pi))[:, None], d.shape[0], axis=1)
    _, dose, _, _, _ = oracle_mod.solve_fixed(ph, xs, d, w, L, ext, inflow, tol=1e-14)
    assert np.allclose(rho * dose, np.dot(E, S), rtol=1e-12, atol=0)
