"""Chained-direction sweeps: the K consecutive directions of one octant swept
back to back by one workgroup (couplings 6 / 7 / 8: 1 / 2 / 4 z layers per
wave), with q and psi in the chain layout.  Every cell's arithmetic is that
of the other schedules, so the dose is identical bit for bit; the boundary
outflows are summed per direction and close the particle balance."""
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


def _run(prob, **kw):
    s = dctsn.Solver(prob)
    try:
        st = s.solve(**kw)
        return st, s.dose()
    finally:
        s.close()


def _ring(n):
    base = I.make_problem("tiny_abd")
    pos, axis = I.ring_sources(n, 360.0 / n)
    return I.Problem(f"tiny_abd_ring{n}", base.phantom, base.xs, base.dirs, base.weights, base.L, pos, axis,
                     base.fan_deg, base.cone_deg, base.group_w)


def test_chained_bitwise_tiny_abd():
    """21 x 19 x 6 abdomen, S6 (6 directions per octant): chains of 2, 3 and 6
    directions with 1, 2 and 4 z layers per wave, FP64 and FP32."""
    prob = I.make_problem("tiny_abd")
    ref = {p: _run(prob, precision=p, tol=1e-8 if p == "fp64" else 1e-6, sweep_bk=16, sweep_sync=2)
           for p in ("fp64", "fp32")}
    for K in (2, 3, 6):
        for cpl in (6, 7, 8):
            for p in ("fp64", "fp32"):
                _say(f"[chain] tiny_abd K={K} coupling={cpl} {p}")
                st, d = _run(prob, precision=p, tol=1e-8 if p == "fp64" else 1e-6, sweep_bk=16, sweep_sync=cpl,
                             sweep_chain=K)
                assert (st.sweep_sync, st.sweep_chain) == (cpl, K)
                assert np.array_equal(st.iters, ref[p][0].iters)
                assert np.array_equal(d, ref[p][1])


def test_chained_bitwise_c2_grid():
    """Full 64 x 64 x 16 grid, S8 (10 directions per octant), two iterations
    per group: chains of 2, 5 and 10 directions against the barrier schedule."""
    prob = I.make_problem("c2")
    fi = np.full(prob.G, 2, dtype=np.int32)
    _, ref = _run(prob, precision="fp32", fixed_iters=fi, sweep_bk=16, sweep_sync=2)
    for K, cpl in ((2, 7), (5, 7), (10, 6), (10, 8)):
        _say(f"[chain] c2 K={K} coupling={cpl} fp32")
        st, d = _run(prob, precision="fp32", fixed_iters=fi, sweep_bk=16, sweep_sync=cpl, sweep_chain=K)
        assert (st.sweep_sync, st.sweep_chain) == (cpl, K)
        assert np.array_equal(d, ref)


def test_chained_batched_sources():
    """Three right-hand sides (sources 120 degrees apart) chained: the same
    dose as the unchained batched solve, bit for bit, and every source keeps
    its own stopping point."""
    prob = _ring(3)
    st0, ref = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=5)
    _say("[chain] ring3 K=3 coupling=7 fp64")
    st, d = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=7, sweep_chain=3)
    assert st.sweep_chain == 3
    assert np.array_equal(st.iters, st0.iters)
    assert np.array_equal(d, ref)


def test_chained_balance():
    """Production = removal + leakage per group at a tight tolerance, with the
    leakage summed per direction by the chained kernel; it agrees with the
    unchained schedule's balance to rounding."""
    prob = I.make_problem("tiny_abd")
    st0, _ = _run(prob, precision="fp64", tol=1e-13, sweep_bk=16, sweep_sync=2)
    st, _ = _run(prob, precision="fp64", tol=1e-13, sweep_bk=16, sweep_sync=7, sweep_chain=6)
    assert st.sweep_chain == 6
    P, R, Lk = st.balance[0].T
    _say(f"[chain balance] max |P - R - L| / P = {np.max(np.abs(P - R - Lk) / P):.2e}")
    assert np.all(np.abs(P - R - Lk) <= 1e-10 * P)
    assert np.allclose(st.balance, st0.balance, rtol=1e-12, atol=0)


def test_chained_fallbacks():
    """Chains need one block, ny <= nx and no kept fluxes: otherwise the solve
    runs the barrier coupling unchained (same dose)."""
    prob = I.make_problem("tiny_abd")
    _, ref = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2)
    st, d = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=7, sweep_chain=3, keep_adjoint=True)
    assert (st.sweep_sync, st.sweep_chain) == (2, 1)
    assert np.array_equal(d, ref)
    # S6 has 6 directions per octant: a chain of 4 would straddle octants
    st, d = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=7, sweep_chain=4)
    assert (st.sweep_sync, st.sweep_chain) == (2, 1)
    assert np.array_equal(d, ref)
    # ny > nx
    ph = I.cylinder_phantom(9, 14, 4, 3.0)
    tall = I.Problem("tall", ph, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis,
                     prob.fan_deg, prob.cone_deg, prob.group_w)
    _, ref_t = _run(tall, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2)
    st, d = _run(tall, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=6, sweep_chain=2)
    assert (st.sweep_sync, st.sweep_chain) == (2, 1)
    assert np.array_equal(d, ref_t)


def test_autotune_with_chains():
    """Asked to (sweep_chain = -1), the tuner times the chained candidates with
    the rest; whatever it picks, the solve is the one every schedule computes."""
    prob = _ring(4)
    st0, ref = _run(prob, precision="fp32", tol=1e-6, sweep_bk=16, sweep_sync=2)
    s = dctsn.Solver(prob)
    try:
        st = s.solve(precision="fp32", tol=1e-6, autotune=True, sweep_chain=-1)
        _say(f"[chain autotune] picked bk={st.sweep_bk} sync={st.sweep_sync} chain={st.sweep_chain}")
        assert st.sweep_chain in (1, 2, 3, 6)
        assert np.array_equal(st.iters, st0.iters)
        assert np.array_equal(s.dose(), ref)
        st2 = s.solve(precision="fp32", tol=1e-6, autotune=True, sweep_chain=-1)
        assert (st2.sweep_sync, st2.sweep_chain) == (st.sweep_sync, st.sweep_chain) and st2.tune_ms == 0
        assert np.array_equal(s.dose(), ref)
    finally:
        s.close()
