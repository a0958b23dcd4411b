"""Source-chained sweeps (couplings 9 / 10: 2 / 1 z layers per wave): one
direction of up to R unfinished right-hand sides swept back to back by one
workgroup, q and psi in the class layouts.  Every cell's arithmetic is that of
the layered-wave schedule, so the dose is identical bit for bit; the boundary
outflows are summed per source and close the particle balance."""
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


def _ring(n, base="tiny_abd", step=None):
    b = I.make_problem(base)
    pos, axis = I.ring_sources(n, 360.0 / n if step is None else step)
    return I.Problem(f"{base}_ring{n}", b.phantom, b.xs, b.dirs, b.weights, b.L, pos, axis, b.fan_deg,
                     b.cone_deg, b.group_w)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs_chained_bitwise_ring(prec):
    """21 x 19 x 6 abdomen, 5 sources 72 degrees apart, S6, converged at tol:
    the sources stop at different iterations, so the chains are rebuilt from
    the unfinished ones as the solve goes on.  Chains of 2, 3, 4 and 8 (more
    than the sources) with 2 and 1 z layers per wave against the layered-wave
    schedule: the same iterations, the same dose bit for bit."""
    prob = _ring(5)
    tol = 1e-8 if prec == "fp64" else 1e-6
    st0, ref = _run(prob, precision=prec, tol=tol, sweep_bk=16, sweep_sync=5)
    assert st0.sweep_sync == 5
    assert len({tuple(r) for r in st0.iters}) > 1        # the sources do finish at different iterations
    for R in (2, 3, 4, 8):
        for cpl in (9, 10):
            _say(f"[rhs chain] ring5 R={R} coupling={cpl} {prec}")
            st, d = _run(prob, precision=prec, tol=tol, sweep_bk=16, sweep_sync=cpl, sweep_rhs_chain=R)
            assert (st.sweep_sync, st.sweep_rhs_chain) == (cpl, R)
            assert np.array_equal(st.iters, st0.iters)
            assert np.array_equal(d, ref)


def test_rhs_chained_c4_grid():
    """The 36-source axial scan (64 x 64 x 16 cylinder, S6, P3), two iterations
    per group: chains of 2, 3, 4, 6 and 8 sources against the layered-wave
    schedule, FP32 and FP64."""
    prob = I.make_problem("c4")
    fi = np.full(prob.G, 2, dtype=np.int32)
    for prec in ("fp32", "fp64"):
        _, ref = _run(prob, precision=prec, fixed_iters=fi, sweep_bk=16, sweep_sync=5)
        for R, cpl in ((2, 9), (3, 9), (4, 9), (6, 10), (8, 9)):
            _say(f"[rhs chain] c4 R={R} coupling={cpl} {prec}")
            st, d = _run(prob, precision=prec, fixed_iters=fi, sweep_bk=16, sweep_sync=cpl, sweep_rhs_chain=R)
            assert (st.sweep_sync, st.sweep_rhs_chain) == (cpl, R)
            assert np.array_equal(d, ref)


def test_rhs_chained_balance():
    """Production = removal + leakage per group and source at a tight
    tolerance, with the leakage summed per source by the chained kernel; it
    agrees with the layered-wave schedule's balance to rounding."""
    prob = _ring(3)
    st0, _ = _run(prob, precision="fp64", tol=1e-13, sweep_bk=16, sweep_sync=5)
    st, _ = _run(prob, precision="fp64", tol=1e-13, sweep_bk=16, sweep_sync=9, sweep_rhs_chain=3)
    assert st.sweep_rhs_chain == 3
    for b in range(prob.B):
        P, R, Lk = st.balance[b].T
        assert np.all(np.abs(P - R - Lk) <= 1e-10 * P)
    _say(f"[rhs chain balance] max |P - R - L| / P = "
         f"{max(np.max(np.abs(bb[:, 0] - bb[:, 1] - bb[:, 2]) / bb[:, 0]) for bb in st.balance):.2e}")
    assert np.allclose(st.balance, st0.balance, rtol=1e-12, atol=0)


def test_rhs_chained_fallbacks():
    """Source chains need several right-hand sides, one block, ny <= nx, no
    kept fluxes and no test inflow: otherwise the solve runs the barrier
    coupling unchained (same dose)."""
    prob = _ring(3)
    _, ref = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2)
    st, d = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=9, sweep_rhs_chain=3, keep_adjoint=True)
    assert (st.sweep_sync, st.sweep_rhs_chain) == (2, 1)
    assert np.array_equal(d, ref)
    one = I.make_problem("tiny_abd")
    _, ref1 = _run(one, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2)
    st, d = _run(one, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=9, sweep_rhs_chain=2)
    assert (st.sweep_sync, st.sweep_rhs_chain) == (2, 1)
    assert np.array_equal(d, ref1)
    # test inflow
    infl = np.linspace(0.1, 0.2, prob.G)
    _, ref_i = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2, test_inflow=infl)
    st, d = _run(prob, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=9, sweep_rhs_chain=3, test_inflow=infl)
    assert (st.sweep_sync, st.sweep_rhs_chain) == (2, 1)
    assert np.array_equal(d, ref_i)
    # ny > nx
    ph = I.cylinder_phantom(9, 14, 4, 3.0)
    tall = I.Problem("tall", ph, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis,
                     prob.fan_deg, prob.cone_deg, prob.group_w)
    _, ref_t = _run(tall, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=2)
    st, d = _run(tall, precision="fp64", tol=1e-8, sweep_bk=16, sweep_sync=10, sweep_rhs_chain=2)
    assert (st.sweep_sync, st.sweep_rhs_chain) == (2, 1)
    assert np.array_equal(d, ref_t)


def test_rhs_chained_adjoint_after_forward():
    """A forward solve that keeps its fluxes for the adjoint cannot run on
    source chains: asked for them, it runs the barrier coupling, and the
    adjoint after it gives the gradient of a barrier-coupled forward."""
    prob = _ring(2)
    roi = np.zeros(prob.phantom.C)
    roi[prob.phantom.C // 2] = 1.0
    fi = np.full(prob.G, 3, dtype=np.int32)
    out = []
    for cpl, R in ((2, 0), (9, 2)):
        s = dctsn.Solver(prob)
        try:
            st = s.solve(precision="fp64", fixed_iters=fi, keep_adjoint=True, sweep_bk=16, sweep_sync=cpl,
                         sweep_rhs_chain=R)
            assert st.sweep_sync == 2
            out.append(s.adjoint(roi, fixed_iters=fi))
        finally:
            s.close()
    # the ray back-projection sums with FP64 atomics: equal up to their order
    for x, y in ((out[0].d_density, out[1].d_density), (out[0].d_group_w, out[1].d_group_w)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_autotune_with_rhs_chains():
    """The tuner times the source chains with the other candidates; whatever
    it picks, the solve is the one every schedule computes."""
    prob = _ring(6)
    st0, ref = _run(prob, precision="fp32", tol=1e-6, sweep_bk=16, sweep_sync=5)
    s = dctsn.Solver(prob)
    try:
        st = s.solve(precision="fp32", tol=1e-6, autotune=True)
        _say(f"[rhs chain autotune] picked bk={st.sweep_bk} sync={st.sweep_sync} chain={st.sweep_chain} "
             f"sources={st.sweep_rhs_chain}")
        assert st.sweep_rhs_chain in (1, 2, 3, 4, 6)
        assert np.array_equal(st.iters, st0.iters)
        assert np.array_equal(s.dose(), ref)
        st2 = s.solve(precision="fp32", tol=1e-6, autotune=True)
        assert (st2.sweep_sync, st2.sweep_rhs_chain) == (st.sweep_sync, st.sweep_rhs_chain) and st2.tune_ms == 0
        assert np.array_equal(s.dose(), ref)
    finally:
        s.close()


def test_rhs_chain_argument_checks():
    prob = _ring(3)
    s = dctsn.Solver(prob)
    try:
        for kw in ({"sweep_rhs_chain": 9}, {"sweep_rhs_chain": -1}, {"sweep_sync": 11}):
            with pytest.raises(dctsn.DctError) as e:
                s.solve(precision="fp64", **kw)
            assert e.value.code == dctsn.DCT_EINVAL
    finally:
        s.close()
