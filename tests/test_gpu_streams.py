"""Iteration sets split over two streams (rhs_streams): the right-hand sides
fall in two halves whose transition, fused and sweep launches run on two
streams, so that one half's sweep overlaps the other half's fused kernel.
The halves share no data, so every result equals the one-stream solve bit
for bit; the FP64 result also matches the oracle."""
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
        return st, s.dose(), s.moments()
    finally:
        s.close()


def _ring(n):
    base = I.make_problem("tiny_abd")
    pos, axis = I.ring_sources(n, 360.0 / n)
    return I.Problem(f"tiny_abd_ring{n}", base.phantom, base.xs, base.dirs, base.weights, base.L, pos, axis,
                     base.fan_deg, base.cone_deg, base.group_w)


@pytest.mark.parametrize("prec,cpl,R", [("fp32", 5, 0), ("fp64", 5, 0), ("fp32", 4, 0), ("fp64", 10, 2),
                                        ("fp32", 9, 3)])
def test_two_streams_bitwise_converged(prec, cpl, R):
    """Five sources (halves of 2 and 3), each stopping on its own test;
    layered waves and chained sources."""
    prob = _ring(5)
    tol = 1e-8 if prec == "fp64" else 1e-6
    kw = dict(precision=prec, tol=tol, fuse_maps=1, sweep_bk=16, sweep_sync=cpl, sweep_rhs_chain=R)
    st1, d1, m1 = _run(prob, rhs_streams=1, **kw)
    st2, d2, m2 = _run(prob, rhs_streams=2, profile=2, **kw)
    _say(f"[streams] ring5 {prec} coupling {cpl}: streams {st1.rhs_streams} / {st2.rhs_streams}, "
         f"iterations {int(st2.iters.sum())}, timed sweeps {st2.sweep_launches}, fused {st2.fused_launches}")
    assert st1.rhs_streams == 1 and st2.rhs_streams == 2
    assert st2.fused_maps == 1 and st2.sweep_sync == cpl and st2.sweep_rhs_chain == max(R, 1)
    assert np.array_equal(st2.iters, st1.iters)
    assert np.array_equal(st2.eps, st1.eps)
    assert np.array_equal(d2, d1) and np.array_equal(m2, m1)
    assert st2.sweep_launches > 0 and st2.sweep_ms > 0 and st2.fused_launches > 0
    # every iteration set launches one sweep per half
    assert st1.sweep_launches_all == st1.iteration_sets and st2.sweep_launches_all == 2 * st2.iteration_sets


def test_two_streams_match_oracle():
    import oracle

    prob = _ring(3)
    ref = oracle.solve_problem(prob, tol=1e-10)
    fi = ref.iters.max(0)
    ref = oracle.solve_problem(prob, fixed_iters=fi)
    st, d, _ = _run(prob, precision="fp64", fixed_iters=fi, fuse_maps=1, sweep_bk=16, sweep_sync=5, rhs_streams=2)
    assert st.rhs_streams == 2
    e = float(np.abs(d - ref.dose).max() / np.abs(ref.dose).max())
    _say(f"[streams] ring3 fp64 two streams vs oracle: dose rel err {e:.2e}")
    assert e < 1e-10


def test_two_streams_c4_default():
    """The 36-source axial scan, converged in FP32: by default the iteration
    sets run on two streams; the same iterations and dose as one stream."""
    prob = I.make_problem("c4")
    st1, d1, _ = _run(prob, precision="fp32", tol=prob.tol, sweep_bk=16, sweep_sync=5, rhs_streams=1)
    st2, d2, _ = _run(prob, precision="fp32", tol=prob.tol, sweep_bk=16, sweep_sync=5)
    _say(f"[streams] c4 fp32: one stream {st1.solve_ms:.1f} ms, default ({st2.rhs_streams} streams) "
         f"{st2.solve_ms:.1f} ms, {int(st2.iters.sum())} iterations")
    assert st1.rhs_streams == 1 and st2.rhs_streams == 2 and st2.fused_maps == 1
    assert np.array_equal(st2.iters, st1.iters)
    assert np.array_equal(d2, d1)


def test_two_streams_c4_chained_sources_fp64():
    """The 36-source scan in FP64 on chains of 8 sources (the tuner's choice
    on one stream), two iterations per group: by default two streams, each
    half's launches on 5 chains of 4 sources per direction; bitwise one stream."""
    prob = I.make_problem("c4")
    fi = np.full(prob.G, 2, dtype=np.int32)
    kw = dict(precision="fp64", fixed_iters=fi, sweep_bk=16, sweep_sync=10, sweep_rhs_chain=8)
    st1, d1, _ = _run(prob, rhs_streams=1, **kw)
    st2, d2, _ = _run(prob, **kw)
    _say(f"[streams] c4 fp64 chained sources: one stream {st1.solve_ms:.1f} ms, default ({st2.rhs_streams} "
         f"streams) {st2.solve_ms:.1f} ms")
    assert st1.rhs_streams == 1 and st2.rhs_streams == 2 and st2.sweep_rhs_chain == 8
    assert np.array_equal(d2, d1)


def test_two_streams_fallbacks():
    """Two streams only with the fused kernel, no graph, and layered waves
    (B >= 2) or chained sources (B >= 4); otherwise one stream with the same
    results."""
    prob = _ring(4)
    fi = np.full(prob.G, 3, dtype=np.int32)
    base = dict(precision="fp32", fixed_iters=fi, sweep_bk=16, rhs_streams=2)
    st0, d0, _ = _run(prob, fuse_maps=1, sweep_sync=5, rhs_streams=1, precision="fp32", fixed_iters=fi)
    for kw in ({"fuse_maps": 1, "sweep_sync": 5, "use_graph": True}, {"fuse_maps": 1, "sweep_sync": 2},
               {"fuse_maps": -1, "sweep_sync": 5}, {"fuse_maps": 1, "sweep_sync": 6, "sweep_chain": 2}):
        st, d, _ = _run(prob, **base, **kw)
        _say(f"[streams] fallback {kw}: streams {st.rhs_streams}")
        assert st.rhs_streams == 1
        assert np.array_equal(d, d0)
    st, d, _ = _run(prob, **base, fuse_maps=1, sweep_sync=10, sweep_rhs_chain=2)
    assert st.rhs_streams == 2 and np.array_equal(d, d0)
    three = _ring(3)
    _, d3, _ = _run(three, fuse_maps=1, sweep_sync=5, rhs_streams=1, precision="fp32", fixed_iters=fi)
    st, d, _ = _run(three, **base, fuse_maps=1, sweep_sync=10, sweep_rhs_chain=2)
    assert st.rhs_streams == 1 and st.sweep_sync == 10 and np.array_equal(d, d3)
    one = I.make_problem("tiny_abd")
    st, _, _ = _run(one, precision="fp32", fixed_iters=fi, fuse_maps=1, sweep_bk=16, sweep_sync=5, rhs_streams=2)
    assert st.rhs_streams == 1
    s = dctsn.Solver(prob)
    try:
        with pytest.raises(dctsn.DctError) as e:
            s.solve(precision="fp32", fixed_iters=fi, rhs_streams=3)
        assert e.value.code == dctsn.DCT_EINVAL
    finally:
        s.close()
