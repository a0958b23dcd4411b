"""The allocation-free effective-dose entry point (dct_effective_dose_noalloc)
against dct_effective_dose on the same solve: two calls in a row on one GPU,
the second on a smaller problem (fewer groups, materials and voxels), so the
second call finds the fixed scratch holding the first call's larger table."""
import numpy as np
import pytest

from paper_1811_12391_amd import dctsn, inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dctsn.lib()
    yield


def _table(seed):
    rng = np.random.default_rng(seed)
    E = np.linspace(15.0, 110.0, 9)
    return E, rng.uniform(0.5, 4.0, E.size)


def _case(name, precision, summed, with_zero, seed):
    import torch

    prob = I.make_problem(name)
    ph = prob.phantom
    s = dctsn.Solver(prob)
    try:
        s.solve(precision=precision, fixed_iters=np.full(prob.G, 3, np.int32))
        E, f = _table(seed)
        zm = None
        if with_zero:
            zm = np.zeros(len(ph.material_names), dtype=np.uint8)
            zm[ph.material_names.index("air")] = 1
        want = s.effective_dose(E, f, zero_material=zm, summed=summed)
        out = torch.full(want.shape, -1.0, dtype=torch.float64, device="cuda")
        dctsn.effective_dose_noalloc(s.h, E, f, out, zero_material=zm, summed=summed)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        s.close()
    print(f"[noalloc] {name} {precision} summed={summed} zero={with_zero}: G={prob.G} C={ph.C} "
          f"max|diff|={np.abs(got - want).max():.3e}", flush=True)
    return got, want


def test_noalloc_matches_effective_dose_two_calls():
    # first call: 5 groups, 5 materials (air zeroed), per right-hand side
    got, want = _case("tiny_abd", "fp64", False, True, 11)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    # second call, smaller: 3 groups, 2 materials, summed over sources, no
    # zero flags (the scratch still holds the first call's 5 factors and flags)
    got, want = _case("tiny", "fp32", True, False, 12)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_noalloc_needs_a_solve():
    import torch

    prob = I.make_problem("tiny")
    s = dctsn.Solver(prob)
    try:
        E, f = _table(1)
        out = torch.zeros(prob.phantom.C, dtype=torch.float64, device="cuda")
        with pytest.raises(dctsn.DctError) as e:
            dctsn.effective_dose_noalloc(s.h, E, f, out, summed=True)
        assert e.value.code == dctsn.DCT_ESTATE
        s.solve(precision="fp64", fixed_iters=np.full(prob.G, 2, np.int32))
        with pytest.raises(dctsn.DctError) as e:
            dctsn.effective_dose_noalloc(s.h, E[::-1], f, out, summed=True)
        assert e.value.code == dctsn.DCT_EINVAL
    finally:
        s.close()
