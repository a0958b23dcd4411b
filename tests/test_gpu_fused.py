"""The fused iteration kernel (direction->moment map, combine and
moment->direction map of every iteration in one kernel per slab, moments and
the next source kept in LDS) against the separate kernels: the same
arithmetic in the same order, so the same iterations and dose bit for bit;
and against the oracle directly."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_bitwise_tiny_abd(prec):
    """21 x 19 x 6 abdomen (ragged slabs: 19 y rows), S6, P3, converged."""
    prob = I.make_problem("tiny_abd")
    tol = 1e-8 if prec == "fp64" else 1e-6
    st0, d0, m0 = _run(prob, precision=prec, tol=tol, fuse_maps=-1, sweep_bk=16, sweep_sync=2)
    _say(f"[fused] tiny_abd {prec}")
    st, d, m = _run(prob, precision=prec, tol=tol, fuse_maps=1, sweep_bk=16, sweep_sync=2)
    assert st0.fused_maps == 0 and st.fused_maps == 1
    assert np.array_equal(st.iters, st0.iters)
    assert np.array_equal(d, d0) and np.array_equal(m, m0)


def test_fused_batched_and_chained():
    """Three right-hand sides; fused maps with and without chained sweeps."""
    prob = _ring(3)
    st0, d0, _ = _run(prob, precision="fp32", tol=1e-6, fuse_maps=-1, sweep_bk=16, sweep_sync=5)
    for cpl, K in ((5, 1), (7, 3), (6, 6)):
        _say(f"[fused] ring3 coupling={cpl} chain={K}")
        st, d, _ = _run(prob, precision="fp32", tol=1e-6, fuse_maps=1, sweep_bk=16, sweep_sync=cpl, sweep_chain=K)
        assert st.fused_maps == 1 and st.sweep_chain == K
        assert np.array_equal(st.iters, st0.iters)
        assert np.array_equal(d, d0)


def test_fused_c2_grid_s8():
    """Full 64 x 64 x 16 grid, S8 (40 directions per class: two psi load
    rounds per row), two iterations per group, FP32 and FP64."""
    prob = I.make_problem("c2")
    fi = np.full(prob.G, 2, dtype=np.int32)
    for prec in ("fp32", "fp64"):
        _say(f"[fused] c2 {prec}")
        _, d0, _ = _run(prob, precision=prec, fixed_iters=fi, fuse_maps=-1, sweep_bk=16, sweep_sync=2)
        st, d, _ = _run(prob, precision=prec, fixed_iters=fi, fuse_maps=1, sweep_bk=16, sweep_sync=2)
        assert st.fused_maps == 1
        assert np.array_equal(d, d0)


def test_fused_c4_persistent_items():
    """The 36-source axial scan, two iterations per group: 2,304 slabs over
    the persistent workgroups (several each, paired on XCDs), the
    first-iteration form at every group start; bitwise the separate kernels,
    FP32 and FP64, and the default picks the fused kernel."""
    prob = I.make_problem("c4")
    fi = np.full(prob.G, 2, dtype=np.int32)
    for prec in ("fp32", "fp64"):
        _say(f"[fused] c4 {prec}")
        d0, d = [], []
        for fm, out in ((-1, d0), (0, d)):
            s = dctsn.Solver(prob)
            try:
                st = s.solve(precision=prec, fixed_iters=fi, fuse_maps=fm, sweep_bk=16, sweep_sync=5)
                out.append(s.dose())
            finally:
                s.close()
        assert st.fused_maps == 1
        assert np.array_equal(d[0], d0[0])


def test_fused_matches_oracle():
    import oracle

    prob = I.make_problem("tiny")
    ref = oracle.solve_problem(prob, tol=1e-10)
    fi = ref.iters.max(0)
    ref = oracle.solve_problem(prob, fixed_iters=fi)
    st, d, _ = _run(prob, precision="fp64", fixed_iters=fi, fuse_maps=1)
    assert st.fused_maps == 1
    e = float(np.abs(d - ref.dose).max() / np.abs(ref.dose).max())
    _say(f"[fused] tiny fp64 vs oracle: dose rel err {e:.2e}")
    assert e < 1e-10


def test_fused_fallback_bf16():
    prob = I.make_problem("tiny_abd")
    fi = np.full(prob.G, 3, dtype=np.int32)
    st0, d0, _ = _run(prob, precision="fp32_bf16map", fixed_iters=fi, fuse_maps=-1)
    st, d, _ = _run(prob, precision="fp32_bf16map", fixed_iters=fi, fuse_maps=1)
    assert st.fused_maps == 0
    assert np.array_equal(d, d0)
