"""Pins of the oracle adjoint (gradient of ROI dose with respect to voxel
densities and source group weights): transposition identities of its linear
blocks and central finite differences of the full forward solve."""
import numpy as np
import pytest

from paper_1811_12391_amd import inputs as I


def test_frozen_sweep_dot_product(oracle_mod):
    """<s, L_F q> = <L_F^T s, q> for the sweep with a frozen fixup set F taken
    from a sweep that fixed many faces (optically thick cells)."""
    rng = np.random.default_rng(11)
    nx, ny, nz = 6, 5, 4
    C = nx * ny * nz
    sig = rng.uniform(0.1, 8.0, C)
    d, w = I.lq_quadrature(4)
    q0 = rng.uniform(0, 1, (24, C)) * (rng.uniform(size=(24, C)) < 0.3)
    _, mask = oracle_mod.sweep_masked((nx, ny, nz), (1.0, 1.2, 0.8), sig, d, q0)
    assert (mask > 0).sum() > 100
    for _ in range(3):
        q = rng.standard_normal((24, C))
        s = rng.standard_normal((24, C))
        psi, _ = oracle_mod.sweep_masked((nx, ny, nz), (1.0, 1.2, 0.8), sig, d, q, mask_in=mask)
        lam = oracle_mod.sweep_adjoint((nx, ny, nz), (1.0, 1.2, 0.8), sig, d, s, mask)
        a, b = np.sum(s * psi), np.sum(lam * q)
        assert abs(a - b) <= 1e-12 * (abs(a) + np.abs(s * psi).sum())


def test_frozen_sweep_matches_deciding_sweep(oracle_mod):
    """Freezing the fixup at the sets a sweep chose reproduces that sweep."""
    rng = np.random.default_rng(12)
    nx, ny, nz = 5, 6, 3
    C = nx * ny * nz
    sig = rng.uniform(0.1, 10.0, C)
    d, w = I.lq_quadrature(6)
    q = rng.uniform(0, 1, (48, C)) * (rng.uniform(size=(48, C)) < 0.4)
    psi, mask = oracle_mod.sweep_masked((nx, ny, nz), (1.0, 1.0, 1.0), sig, d, q)
    psi2, _ = oracle_mod.sweep_masked((nx, ny, nz), (1.0, 1.0, 1.0), sig, d, q, mask_in=mask)
    assert np.allclose(psi, psi2, rtol=1e-13, atol=1e-16)


def _abd_small():
    ph = I.abdomen_phantom(10, 9, 4, 3.6)
    xs = I.xs_tables(ph.material_names, 3, 1)
    d, w = I.lq_quadrature(4)
    pos, ax = I.top_source()
    gw = I.kramers_weights(xs.edges)
    roi = np.zeros(ph.C)
    roi.reshape(4, 9, 10)[1:3, 3:6, 3:7] = 1.0 / 24
    return I.Problem("abd_small", ph, xs, d, w, 1, pos, ax, 60.0, 40.0, gw), roi


def _R(oracle_mod, prob, roi, rho=None, gw=None, fixup=True):
    ph = prob.phantom
    p2 = I.Phantom(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material,
                   ph.density if rho is None else rho, ph.material_names)
    r = oracle_mod.solve(p2, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis, prob.fan_deg,
                         prob.cone_deg, prob.group_w if gw is None else gw, tol=1e-13, fixup=fixup)
    return float(np.sum(roi * r.dose.sum(0)))


@pytest.mark.parametrize("fixup", [False, True])
def test_adjoint_density_finite_differences(oracle_mod, fixup):
    """dR/drho_v from the adjoint equals central differences of the forward
    solve (tolerance 1e-13) on voxels in the ROI, on the beam path, in bone,
    lung, fat and air."""
    prob, roi = _abd_small()
    ph = prob.phantom
    a = oracle_mod.adjoint_problem(prob, roi, tol=1e-13, fixup=fixup)
    assert abs(a.R - _R(oracle_mod, prob, roi, fixup=fixup)) <= 1e-13 * abs(a.R)
    rng = np.random.default_rng(13)
    picks = []
    for m in range(5):
        ids = np.nonzero(ph.material == m)[0]
        picks += list(rng.choice(ids, min(2, len(ids)), replace=False))
    picks += list(np.nonzero(roi > 0)[0][:3])
    for v in picks:
        h = 1e-4 * max(ph.density[v], 1e-2)
        r1, r2 = ph.density.copy(), ph.density.copy()
        r1[v] += h
        r2[v] -= h
        fd = (_R(oracle_mod, prob, roi, rho=r1, fixup=fixup) - _R(oracle_mod, prob, roi, rho=r2, fixup=fixup)) / (2 * h)
        assert abs(fd - a.d_density[v]) <= 1e-6 * abs(fd) + 1e-9 * abs(a.R), (v, fd, a.d_density[v])


def test_adjoint_group_weights_exact(oracle_mod):
    """Without the fixup the solve is linear in the group weights, so a
    one-sided difference is exact up to rounding.  (With the fixup it is only
    piecewise linear: changing the group mix can flip fixed faces.)"""
    prob, roi = _abd_small()
    a = oracle_mod.adjoint_problem(prob, roi, tol=1e-13, fixup=False)
    base = _R(oracle_mod, prob, roi, fixup=False)
    for g in range(prob.G):
        gw = prob.group_w.copy()
        gw[g] += 1e-2
        fd = (_R(oracle_mod, prob, roi, gw=gw, fixup=False) - base) / 1e-2
        assert abs(fd - a.d_group_w[g]) <= 1e-9 * abs(a.d_group_w).max()
