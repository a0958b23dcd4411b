"""GPU superposed sources (several beams in one collided solve, the CT-scan
form of Sec. III-C) against the FP64 oracle's superposed solve, and the
exact doubling identity on the device."""
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
    return float(np.abs(a - b).max() / np.abs(b).max())


def l2rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("S", [4, 2])
def test_superposed_fp64_matches_oracle(S):
    import oracle

    prob = I.make_problem("tiny_ct")
    ref0 = oracle.solve_problem(prob, tol=1e-10, superpose=S)
    fi = ref0.iters.max(0)
    ref = oracle.solve_problem(prob, fixed_iters=fi, superpose=S)
    _say(f"[superpose fp64] tiny_ct S={S} iters {fi.tolist()}")
    s = dctsn.Solver(prob)
    try:
        st = s.solve(precision="fp64", fixed_iters=fi, superpose=S)
        dose, pu, pc = s.dose(want_phi=True)
    finally:
        s.close()
    assert dose.shape == (prob.B // S, prob.phantom.C)
    assert np.array_equal(st.iters, np.broadcast_to(fi, st.iters.shape))
    assert rel(pu, ref.phi_u) < 1e-12
    e_pc, e_dose = rel(pc, ref.phi[:, :, 0]), rel(dose, ref.dose)
    _say(f"[superpose fp64] S={S}: phi_c rel err {e_pc:.2e}, dose rel err {e_dose:.2e}")
    assert e_pc < 1e-10
    assert e_dose < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_superposed_doubling_exact(precision):
    """Two copies of a beam superposed give exactly twice the single-beam
    solve on the device too (every input of the collided solve doubles)."""
    prob = I.make_problem("tiny")
    two = I.Problem("tiny2", prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L,
                    np.repeat(prob.src_pos, 2, 0), np.repeat(prob.src_axis, 2, 0), prob.fan_deg, prob.cone_deg,
                    prob.group_w)
    s1, s2 = dctsn.Solver(prob), dctsn.Solver(two)
    try:
        a = s1.solve(precision=precision)
        d1 = s1.dose()
        b = s2.solve(precision=precision, superpose=2)
        d2 = s2.dose()
    finally:
        s1.close()
        s2.close()
    assert np.array_equal(a.iters, b.iters)
    assert np.array_equal(d2, 2.0 * d1)


def test_ct16_fp32_vs_oracle_two_iterations():
    """Full-size CT-scan form: 16 cone beams of 30 degrees around the 64x64x16
    cylinder, superposed into one FP32 solve (autotuned sweep schedule, graph
    replay), two source iterations per group on both sides."""
    import oracle

    prob = I.make_problem("ct16")
    fi = np.full(prob.G, 2, dtype=np.int32)
    _say("[ct16] oracle, superposed, 2 iterations per group")
    ref = oracle.solve_problem(prob, fixed_iters=fi, superpose=16)
    s = dctsn.Solver(prob)
    try:
        _say("[ct16] GPU fp32")
        s.solve(precision="fp32", fixed_iters=fi, superpose=16, autotune=True, use_graph=True)
        dose = s.dose()
    finally:
        s.close()
    err = l2rel(dose, ref.dose)
    _say(f"[ct16] dose L2 rel err {err:.3e}")
    assert dose.shape == (1, prob.phantom.C)
    assert err <= 1e-4


def test_superpose_argument_errors():
    prob = I.make_problem("tiny_ct")
    s = dctsn.Solver(prob)
    try:
        for kw in (dict(superpose=3), dict(superpose=-1), dict(superpose=2, keep_adjoint=True)):
            with pytest.raises((dctsn.DctError, ValueError)) as e:
                s.solve(precision="fp64", **kw)
            if isinstance(e.value, dctsn.DctError):
                assert e.value.code == dctsn.DCT_EINVAL
        # the library itself rejects what the binding would pass through
        o = dctsn.dct_opts()
        o.precision, o.tol, o.max_iter, o.fixup, o.superpose = 0, 1e-6, 10, 1, 3
        assert dctsn.lib().dct_solve(s.h, dctsn.ct.byref(o), None) == dctsn.DCT_EINVAL
    finally:
        s.close()


def test_superposed_schedules_and_roi_dose():
    """Superposed right-hand sides through every single-block schedule (layered
    waves, chained sources, fused maps on and off) give the same dose bit for
    bit, and the library's ROI response equals roi . summed dose."""
    prob = I.make_problem("tiny_ct")
    S = 2
    fi = np.full(prob.G, 3, dtype=np.int32)
    roi = np.zeros(prob.phantom.C)
    roi[prob.phantom.C // 3: prob.phantom.C // 3 + 40] = 0.025
    ref = None
    for kw in ({"sweep_sync": 2, "fuse_maps": -1}, {"sweep_sync": 5, "fuse_maps": 1},
               {"sweep_sync": 9, "sweep_rhs_chain": 2, "fuse_maps": 1},
               {"sweep_sync": 10, "sweep_rhs_chain": 3, "fuse_maps": -1}):
        s = dctsn.Solver(prob)
        try:
            st = s.solve(precision="fp32", fixed_iters=fi, superpose=S, sweep_bk=16, **kw)
            d = s.dose()
            R = dctsn.roi_dose(s.h, prob.phantom.C, roi)
        finally:
            s.close()
        _say(f"[superpose schedules] {kw}: ran coupling {st.sweep_sync}, sources per chain {st.sweep_rhs_chain}, "
             f"fused {st.fused_maps}")
        assert st.sweep_sync == kw["sweep_sync"]
        Rh = float(np.dot(roi, d.sum(0)))
        assert abs(R - Rh) <= 1e-12 * abs(Rh)
        if ref is None:
            ref = d
        else:
            assert np.array_equal(d, ref)

