"""Warm-started solves (every group's source iteration starting from the
moments the previous solve on the context left): they converge to the same
discrete fixed point as a cold solve (checked against the oracle at tol
1e-12), and take fewer iterations when the previous solve is close (a
perturbed density, the next source position of a scan)."""
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
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_warm_resolve_same_problem():
    """Re-solving the same problem from its own converged moments stops after
    one iteration per group, within tol of the cold solve."""
    prob = I.make_problem("tiny_abd")
    s = dctsn.Solver(prob)
    try:
        st0 = s.solve(precision="fp64", tol=1e-8)
        d0 = s.dose()
        assert st0.warm_start == 0
        st1 = s.solve(precision="fp64", tol=1e-8, warm_start=True)
        d1 = s.dose()
        _say(f"[warm] same problem: cold {int(st0.iters.sum())} iterations, warm {int(st1.iters.sum())}")
        assert st1.warm_start == 1
        assert np.all(st1.iters == 1)
        assert rel(d1, d0) < 1e-7
        # a different precision does not warm start
        st2 = s.solve(precision="fp32", tol=1e-6, warm_start=True)
        assert st2.warm_start == 0
    finally:
        s.close()


@pytest.mark.parametrize("fuse", [-1, 1])
def test_warm_perturbed_density_matches_oracle(fuse):
    """Densities perturbed by 1%: the warm solve from the unperturbed moments
    and the oracle's cold solve of the perturbed problem agree at tol 1e-12
    (the same fixed point), with fewer iterations than a cold GPU solve."""
    import oracle

    prob = I.make_problem("tiny_abd")
    ph = prob.phantom
    rng = np.random.default_rng(5)
    rho2 = ph.density * (1.0 + 0.01 * rng.standard_normal(ph.C))
    rho2 = np.maximum(rho2, 0.0)
    s = dctsn.Solver(prob)
    try:
        s.solve(precision="fp64", tol=1e-12, fuse_maps=fuse)
        s.set_density(rho2)
        stw = s.solve(precision="fp64", tol=1e-12, warm_start=True, fuse_maps=fuse)
        dw = s.dose()
        stc = s.solve(precision="fp64", tol=1e-12, fuse_maps=fuse)
        dc = s.dose()
    finally:
        s.close()
    assert stw.warm_start == 1 and stc.warm_start == 0
    import dataclasses

    prob2 = dataclasses.replace(prob, phantom=dataclasses.replace(ph, density=rho2))
    ref = oracle.solve_problem(prob2, tol=1e-12)
    ew, ec = rel(dw, ref.dose), rel(dc, ref.dose)
    _say(f"[warm fuse={fuse}] perturbed density: warm {int(stw.iters.sum())} iterations (dose rel err vs oracle "
         f"{ew:.1e}), cold {int(stc.iters.sum())} ({ec:.1e})")
    assert ew < 1e-10 and ec < 1e-10
    assert stw.iters.sum() < stc.iters.sum()


def test_warm_scan_positions():
    """A scan solved one position after the other (sources 10 degrees apart):
    starting each position from the previous one's moments saves iterations
    and gives the cold doses within tol."""
    base = I.make_problem("tiny_abd")
    pos, axis = I.ring_sources(6, 10.0)
    tot = {}
    doses = {}
    for warm in (False, True):
        s = dctsn.Solver(base)
        try:
            n_it, ds = 0, []
            for p in range(6):
                dctsn.set_source(s.h, 1, pos[p:p + 1], axis[p:p + 1], base.fan_deg, base.cone_deg, base.group_w)
                st = s.solve(precision="fp64", tol=1e-8, warm_start=warm)
                assert st.warm_start == (1 if (warm and p > 0) else 0)
                n_it += int(st.iters.sum())
                ds.append(s.dose()[0])
            tot[warm], doses[warm] = n_it, np.array(ds)
        finally:
            s.close()
    _say(f"[warm] 6 scan positions: cold {tot[False]} iterations, warm {tot[True]}")
    assert tot[True] < tot[False]
    assert rel(doses[True], doses[False]) < 1e-6
