"""Persisted sweep schedules (DCT_TUNE_CACHE): a tuned solve appends its
schedule to the file; a new context on the same kind of device starts from
the file and does not tune again; the last entry of a shape wins."""
import os
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


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("DCT_TUNE_CACHE", str(path))
    prob = I.make_problem("tiny_abd")
    fi = np.full(prob.G, 3, dtype=np.int32)
    kw = dict(precision="fp32", fixed_iters=fi, autotune=True)
    a = dctsn.Solver(prob)
    try:
        sa = a.solve(**kw)
        da = a.dose()
    finally:
        a.close()
    lines = path.read_text().splitlines()
    _say(f"[tune cache] {lines}")
    assert sa.tune_ms > 0 and len(lines) == 1
    f = lines[0].split()
    assert f[0] == "dctsn-tune-1" and [int(x) for x in f[3:8]] == [prob.phantom.nx, prob.phantom.ny,
                                                                    prob.phantom.nz, prob.N, prob.B]
    assert [int(x) for x in f[11:14]] == [sa.sweep_sync, sa.sweep_chain, sa.sweep_rhs_chain]
    # a new context starts from the file: no tuning, the same schedule and dose
    b = dctsn.Solver(prob)
    try:
        sb = b.solve(**kw)
        assert sb.tune_ms == 0
        assert (sb.sweep_bk, sb.sweep_sync, sb.sweep_chain) == (sa.sweep_bk, sa.sweep_sync, sa.sweep_chain)
        assert np.array_equal(b.dose(), da)
    finally:
        b.close()
    assert len(path.read_text().splitlines()) == 1
    # the last entry of a shape wins; entries of another device kind are ignored
    other = list(f)
    other[1] = "gfx000"
    other[10:14] = ["8", "1", "1", "1"]
    last = list(f)
    last[10:14] = ["16", "2", "1", "1"]
    with open(path, "a") as fh:
        fh.write(" ".join(last) + "\n")
        fh.write(" ".join(other) + "\n")
        fh.write("not a schedule line\n")
    c = dctsn.Solver(prob)
    try:
        sc = c.solve(**kw)
        assert sc.tune_ms == 0 and sc.sweep_sync == 2
        assert np.array_equal(c.dose(), da)        # every schedule computes the same solve
    finally:
        c.close()
