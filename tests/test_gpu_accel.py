"""Anderson-accelerated within-group iterations (depth m on the scalar-flux
moment): the accelerated solve reaches the same discrete fixed point as the
oracle's plain source iteration (both at tol 1e-12), in fewer iterations on
the strongly scattering 4-group problem; right-hand sides stay independent."""
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


def _run(prob, **kw):
    s = dctsn.Solver(prob)
    try:
        st = s.solve(**kw)
        return st, s.dose(), s.moments()
    finally:
        s.close()


_REF = {}


def _oracle(name):
    import oracle

    if name not in _REF:
        _REF[name] = oracle.solve_problem(I.make_problem(name), tol=1e-12)
    return _REF[name]


@pytest.mark.parametrize("name,m", [("c1", 1), ("c1", 2), ("c1", 3), ("tiny_abd", 2)])
def test_accelerated_matches_oracle(name, m):
    prob = I.make_problem(name)
    ref = _oracle(name)
    st0, d0, _ = _run(prob, precision="fp64", tol=1e-12)
    st, d, mom = _run(prob, precision="fp64", tol=1e-12, accel_depth=m)
    e = rel(d, ref.dose)
    em = rel(mom[:, :, 0], ref.phi[:, :, 0])
    _say(f"[accel] {name} m={m}: iterations plain {int(st0.iters.sum())} (oracle {int(ref.iters.sum())}), "
         f"accelerated {int(st.iters.sum())}; dose rel err vs oracle {e:.1e}, phi_00 {em:.1e}")
    assert e < 1e-10 and em < 1e-10
    if name == "c1":
        assert st.iters.sum() < st0.iters.sum()


def test_accelerated_batched_equals_separate():
    base = I.make_problem("tiny_abd")
    pos, axis = I.ring_sources(3, 120.0)
    prob = I.Problem("ring3", base.phantom, base.xs, base.dirs, base.weights, base.L, pos, axis, base.fan_deg,
                     base.cone_deg, base.group_w)
    st, d, _ = _run(prob, precision="fp64", tol=1e-10, accel_depth=2)
    for b in range(3):
        one = I.Problem("one", base.phantom, base.xs, base.dirs, base.weights, base.L, pos[b:b + 1],
                        axis[b:b + 1], base.fan_deg, base.cone_deg, base.group_w)
        st1, d1, _ = _run(one, precision="fp64", tol=1e-10, accel_depth=2)
        assert np.array_equal(st.iters[b], st1.iters[0])
        assert np.array_equal(d[b], d1[0])


def test_accelerated_fp32_and_warm():
    """FP32 with acceleration stays within the dose bar of the FP64 solve; a
    warm start of the accelerated solve reuses the previous moments."""
    prob = I.make_problem("c1")
    ref = _oracle("c1")
    s = dctsn.Solver(prob)
    try:
        st = s.solve(precision="fp32", tol=1e-6, accel_depth=2)
        d = s.dose()
        e = float(np.linalg.norm(d - ref.dose) / np.linalg.norm(ref.dose))
        _say(f"[accel] c1 fp32 m=2: {int(st.iters.sum())} iterations, dose L2 rel err {e:.1e}")
        assert e <= 1e-4
        st2 = s.solve(precision="fp32", tol=1e-6, accel_depth=2, warm_start=True)
        assert st2.warm_start == 1 and st2.iters.sum() < st.iters.sum()
    finally:
        s.close()


def test_accel_argument_check():
    prob = I.make_problem("tiny")
    s = dctsn.Solver(prob)
    try:
        with pytest.raises(dctsn.DctError) as e:
            s.solve(precision="fp64", accel_depth=5)
        assert e.value.code == dctsn.DCT_EINVAL
    finally:
        s.close()
