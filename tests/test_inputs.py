"""Pins for the synthetic input generators (quadrature, cross sections,
spectrum, phantoms).  None of these values come from the HIP library."""
import json
import math
import os

import numpy as np
import pytest

from paper_1811_12391_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _facts():
    with open(os.path.join(GOLD, "paper_facts.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_quadrature_counts_and_norms(N):
    """N(N+2) directions (Sec. II-A eq. 3; Sec. II-D), unit length, sum w = 4 pi."""
    facts = _facts()["directions_per_sn"]
    d, w = I.lq_quadrature(N)
    assert d.shape == (facts[str(N)], 3) == (N * (N + 2), 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15, rtol=0)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    assert np.all(w > 0)


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_quadrature_symmetry(N):
    """Octant reflections and coordinate permutations map the set onto itself
    with equal weights (level symmetry)."""
    d, w = I.lq_quadrature(N)
    n8 = len(w) // 8
    base = d[:n8]
    for o in range(8):
        s = np.array([-1 if o & 1 else 1, -1 if o & 2 else 1, -1 if o & 4 else 1])
        assert np.array_equal(d[o * n8:(o + 1) * n8], base * s)
        assert np.array_equal(w[o * n8:(o + 1) * n8], w[:n8])
    key = {tuple(np.round(p, 14)): wt for p, wt in zip(base, w[:n8])}
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)]:
        for p, wt in zip(base, w[:n8]):
            q = tuple(np.round(p[list(perm)], 14))
            assert q in key and abs(key[q] - wt) < 1e-15


@pytest.mark.parametrize("N", [4, 6, 8])
def test_quadrature_even_moments(N):
    """Even moments sum w mu^(2m) / 4pi = 1/(2m+1) for m = 0..N/2 (the weight
    conditions plus the one that fixes mu1)."""
    d, w = I.lq_quadrature(N)
    for m in range(0, N // 2 + 1):
        for a in range(3):
            val = np.sum(w * d[:, a] ** (2 * m)) / (4 * math.pi)
            assert abs(val - 1.0 / (2 * m + 1)) < 1e-14, (m, a, val)


def test_quadrature_textbook_values():
    """Published 7-digit LQ_N tables: mu1 S4 0.3500212, S6 0.2666355,
    S8 0.2182179; S6 point weights 0.1761263, 0.1572071; S8 point weights
    0.1209877, 0.0907407, 0.0925926 (agreement to the last printed digit, +-2
    units).  Closed forms: S4 mu1^2 = (4 - sqrt 6.4)/12, S8 mu1 = 1/sqrt 21."""
    assert abs(I.lq_mu1(4) - 0.3500212) < 2e-7
    assert abs(I.lq_mu1(6) - 0.2666355) < 2e-7
    assert abs(I.lq_mu1(8) - 0.2182179) < 2e-7
    d6, w6 = I.lq_quadrature(6)
    u6 = sorted(set(np.round(w6[:6] / (math.pi / 2), 12)))
    assert np.allclose(u6, [0.1572071, 0.1761263], atol=2e-7, rtol=0)
    assert abs(I.lq_mu1(4) ** 2 - (4 - math.sqrt(6.4)) / 12) < 1e-15
    assert abs(I.lq_mu1(8) - 1 / math.sqrt(21)) < 1e-15
    d, w = I.lq_quadrature(8)
    ws = sorted(set(np.round(w[:10] / (math.pi / 2), 7)))
    assert ws == [0.0907407, 0.0925926, 0.1209877]


def test_kn_closed_form_vs_integral():
    """Closed-form Klein-Nishina total = 2 pi integral of dsigma/dOmega; low
    energy expansion is the Thomson cross section 8 pi r_e^2 / 3 times
    (1 - 2k + 26 k^2 / 5 + O(k^3)), k = E / m_e c^2."""
    x, wq = np.polynomial.legendre.leggauss(200)
    for E in [10.0, 20.0, 57.3, 100.0, 120.0, 511.0]:
        num = 2 * math.pi * np.sum(wq * I.kn_dsigma_domega(E, x))
        assert abs(num / I.kn_sigma(E) - 1) < 1e-12
    thomson = 8 * math.pi * I.R_E_CM ** 2 / 3
    k = 1.0 / I.ME_C2_KEV
    assert abs(I.kn_sigma(1.0) / thomson - (1 - 2 * k + 5.2 * k * k)) < 2e-7


def test_photo_calibration_and_mfp():
    """Water at 20 keV has mean free path 1.39 cm exactly (Sec. II-D); at
    100 keV the synthetic model gives within 2% of the printed 6.06 cm."""
    facts = _facts()["water_mfp_cm"]
    mu20 = I.mass_atten(20.0, 7.42) * 1.0
    assert abs(1.0 / mu20 - facts["20"]) < 1e-12
    mfp100 = 1.0 / (I.mass_atten(100.0, 7.42) * 1.0)
    assert abs(mfp100 / facts["100"] - 1) < 0.02


def test_transfer_partition_and_structure():
    """Sum over destination groups of s_0 plus the cutoff loss equals the
    group-averaged Klein-Nishina cross section; no upscatter; s_1/s_0 is a mean
    cosine in [-1, 1]; band <= 1 group at G=4 and <= 7 groups at G=19."""
    from scipy.integrate import quad

    for G, band in [(4, 1), (19, 7)]:
        xs = I.xs_tables(["air", "water", "bone"], G, 3)
        for m in range(xs.M):
            s0 = xs.sigma_s[m, 0]
            # independent group average of the closed-form KN cross section
            avg = np.array([
                quad(lambda E: float(I.kn_sigma(E)), xs.edges[g + 1], xs.edges[g], epsabs=0, epsrel=1e-13)[0]
                / (xs.edges[g] - xs.edges[g + 1]) for g in range(G)]) * I.NE_PER_GRAM
            tot = s0.sum(axis=1) + xs.cutoff[m]
            assert np.allclose(tot, avg, rtol=1e-9, atol=0)
            assert np.abs(np.tril(xs.sigma_s[m], -1)).max() == 0.0
            for g in range(G):
                nz = np.nonzero(s0[g])[0]
                assert nz.max() - g <= band
            mc = xs.sigma_s[m, 1].sum(1) / s0.sum(1)
            assert np.all(np.abs(mc) <= 1)
            # Legendre moments of a positive kernel: |s_l| <= s_0
            assert np.all(np.abs(xs.sigma_s[m, 1:]) <= s0[None] * (1 + 1e-12))
            # total exceeds the scattering part (photoelectric > 0)
            assert np.all(xs.sigma_t[m] > s0.sum(1) + xs.cutoff[m])


def test_kramers_closed_form():
    """Group weights are the normalised integral of (E0 - E)/E over each group."""
    edges = I.group_edges(4)
    w = I.kramers_weights(edges)
    from scipy.integrate import quad

    ref = np.array([quad(lambda E: (120.0 - E) / E, lo, hi, epsabs=0, epsrel=1e-13)[0]
                    for hi, lo in zip(edges[:-1], edges[1:])])
    assert np.allclose(w, ref / ref.sum(), rtol=1e-13, atol=0)
    assert abs(w.sum() - 1) < 1e-15


def test_phantom_geometry():
    """Voxel counts of the paper's meshes (Sec. II-D) and the cylinder
    classification by voxel centre."""
    facts = _facts()["meshes"]
    assert facts["fine"][0] * facts["fine"][1] * facts["fine"][2] == facts["fine"][3]
    assert facts["coarse"][0] * facts["coarse"][1] * facts["coarse"][2] == facts["coarse"][3]
    ph = I.cylinder_phantom(64, 64, 16, 0.6)
    assert ph.C == 65536
    x, y, z = ph.centres()
    assert abs(x[0] + x[-1]) < 1e-12 and abs(z[0] + z[-1]) < 1e-12
    X, Y = np.meshgrid(x, y, indexing="xy")
    inside = (X ** 2 + Y ** 2 <= 17.5 ** 2)
    mat = ph.material.reshape(16, 64, 64)
    assert np.array_equal(mat[3] == 1, inside)
    assert np.all(ph.density[ph.material == 1] == 1.0)


def test_abdomen_seeded():
    """The abdomen phantom is deterministic for a seed and holds all materials."""
    a = I.abdomen_phantom(64, 64, 16, 0.6)
    b = I.abdomen_phantom(64, 64, 16, 0.6)
    assert np.array_equal(a.material, b.material) and np.array_equal(a.density, b.density)
    assert set(np.unique(a.material)) == {0, 1, 2, 3, 4}
    nonair = a.material != 0
    nominal = np.array([I.MATERIALS[n][0] for n in I.ABDOMEN_NAMES])[a.material]
    rel = a.density[nonair] / nominal[nonair] - 1
    assert 0.015 < rel.std() < 0.025
    # lungs only in the upper half (z > 0)
    mat = a.material.reshape(16, 64, 64)
    assert not np.any(mat[:8] == 3) and np.any(mat[8:] == 3)


def test_ring_sources():
    pos, axis = I.ring_sources()
    assert pos.shape == (36, 3)
    assert np.allclose(np.linalg.norm(pos, axis=1), 54.0)
    assert np.allclose(axis, -pos / 54.0)
    # positions k and k+9 are 90 degree rotations about z
    R = np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 1]], dtype=float)
    assert np.allclose(pos[9:18], pos[0:9] @ R.T, atol=1e-12)
