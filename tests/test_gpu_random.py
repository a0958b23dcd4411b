"""Seeded random FP64 parity cases: ragged grids (including several y and z
blocks), S4-S8, P0-P3, 2-4 groups, random beam windows and every sweep
schedule, each against the FP64 oracle at the oracle's own per-group
iteration counts."""
import sys

import numpy as np
import pytest

from paper_1811_12391_amd import dctsn, inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dctsn.lib()
    yield


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# (bk, coupling) of each case: every coupling, with block splits
SCHEDULES = [(16, 3), (8, 3), (4, 3), (16, 5), (16, 4), (2, 1), (16, 2), (0, 0)]


def _case(k):
    rng = np.random.default_rng(1811 + 97 * k)
    while True:
        nx, ny, nz = int(rng.integers(3, 70)), int(rng.integers(3, 140)), int(rng.integers(2, 40))
        if nx * ny * nz <= 40000:
            break
    if k < 3:
        # several y and z blocks for the pipelined coupling
        ny, nz = int(rng.integers(65, 100)), int(rng.integers(17, 24))
        nx = int(rng.integers(3, max(4, 40000 // (ny * nz))))
    bk, sync = SCHEDULES[k % len(SCHEDULES)]
    if sync in (4, 5):
        # layered waves need one block: ny <= 64, nz <= 16 <= bk
        ny, nz = min(ny, 64), min(nz, 16)
    d = min(float(rng.uniform(0.4, 3.0)), 90.0 / max(nx, ny, nz))
    if rng.random() < 0.5:
        ph = I.abdomen_phantom(nx, ny, nz, d, seed=int(rng.integers(1, 10**6)))
    else:
        ph = I.cylinder_phantom(nx, ny, nz, d)
    S = int(rng.choice([4, 6, 8]))
    L = int(rng.integers(0, min(3, S // 2) + 1))
    G = int(rng.integers(2, 5))
    xs = I.xs_tables(ph.material_names, G, L)
    dirs, w = I.lq_quadrature(S)
    pos, axis = I.top_source()
    fan, cone = float(rng.uniform(10, 60)), float(rng.uniform(5, 40))
    prob = I.Problem(f"random{k}", ph, xs, dirs, w, L, pos, axis, fan, cone, I.kramers_weights(xs.edges))
    return prob, (bk, sync)


@pytest.mark.parametrize("k", range(8))
def test_random_case_fp64_matches_oracle(k):
    import oracle

    prob, (bk, sync) = _case(k)
    ph = prob.phantom
    _say(f"[random {k}] {ph.nx}x{ph.ny}x{ph.nz} d={ph.dx:.2f} N={prob.N} L={prob.L} G={prob.G} "
         f"fan={prob.fan_deg:.0f} cone={prob.cone_deg:.0f} schedule {bk}:{sync}")
    ref = oracle.solve_problem(prob, tol=1e-6)
    s = dctsn.Solver(prob)
    try:
        st = s.solve(precision="fp64", fixed_iters=ref.iters[0], sweep_bk=bk, sweep_sync=sync)
        dose, pu, _ = s.dose(want_phi=True)
        mom = s.moments()
    finally:
        s.close()
    _say(f"[random {k}] ran {st.sweep_bk}:{st.sweep_sync}, iterations {int(st.iters.sum())}")
    assert np.array_equal(st.iters, ref.iters)
    assert rel(pu, ref.phi_u) < 1e-12
    assert rel(mom, ref.phi) < 1e-10
    assert rel(dose, ref.dose) < 1e-10
