"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side validation returns the documented status codes (host-only
context, no GPU needed, no kernels launched)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1811_12391_amd import dctsn, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "dctsn.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(dct_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = dctsn.lib()
    syms = _header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(dctsn.EXPORTS) == syms


@pytest.fixture()
def host_ctx():
    h = dctsn.create(-1, None)
    yield h
    dctsn.destroy(h)


def test_create_no_gpu_reports_edevice():
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(dctsn.DctError) as e:
        dctsn.create(0, None)
    assert e.value.code == dctsn.DCT_EDEVICE


def test_validation_codes(host_ctx):
    h = host_ctx
    lib = dctsn.lib()
    prob = I.make_problem("tiny")
    ph, xs = prob.phantom, prob.xs
    # geometry
    with pytest.raises(dctsn.DctError) as e:
        dctsn.set_geometry(h, 0, 1, 1, 1.0, 1.0, 1.0, ph.origin, ph.material, ph.density)
    assert e.value.code == dctsn.DCT_EINVAL
    bad = ph.density.copy()
    bad[3] = np.nan
    with pytest.raises(dctsn.DctError):
        dctsn.set_geometry(h, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material, bad)
    dctsn.set_geometry(h, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material, ph.density)
    # a grid of 2^28 voxels would overflow the kernels' 32-bit byte offsets of
    # per-voxel FP64 arrays: rejected before its arrays are read (so
    # one-element arrays suffice here)
    one_m, one_d = np.zeros(1, np.uint8), np.ones(1)
    lib = dctsn.lib()
    rc = lib.dct_set_geometry(h, 1024, 1024, 256, 1.0, 1.0, 1.0, ph.origin.ctypes.data_as(ct.POINTER(ct.c_double)),
                              one_m.ctypes.data_as(ct.POINTER(ct.c_uint8)), one_d.ctypes.data_as(ct.POINTER(ct.c_double)))
    assert rc == dctsn.DCT_EINVAL and "too large" in dctsn.last_error(h)
    rc = lib.dct_set_geometry(h, 4096, 4096, 0, 1.0, 1.0, 1.0, None, None, None)
    assert rc == dctsn.DCT_EINVAL
    dctsn.set_geometry(h, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material, ph.density)
    # source before xs -> ESTATE (needs G)
    with pytest.raises(dctsn.DctError) as e:
        dctsn.set_source(h, 1, prob.src_pos, prob.src_axis, 20.0, 10.0, prob.group_w)
    assert e.value.code == dctsn.DCT_ESTATE
    # upscatter rejected
    ss = xs.sigma_s[:, : prob.L + 1].copy()
    ss[1, 0, 2, 0] = 0.1
    with pytest.raises(dctsn.DctError) as e:
        dctsn.set_xs(h, xs.G, xs.edges, xs.M, prob.L, xs.sigma_t, ss, xs.kerma)
    assert e.value.code == dctsn.DCT_EINVAL and "upscatter" in str(e.value)
    dctsn.set_xs(h, xs.G, xs.edges, xs.M, prob.L, xs.sigma_t, xs.sigma_s[:, : prob.L + 1], xs.kerma)
    # quadrature: non-unit direction
    d = prob.dirs.copy()
    d[0] *= 1.1
    with pytest.raises(dctsn.DctError):
        dctsn.set_quadrature(h, prob.N, d, prob.weights)
    dctsn.set_quadrature(h, prob.N, prob.dirs, prob.weights)
    # source angles
    with pytest.raises(dctsn.DctError):
        dctsn.set_source(h, 1, prob.src_pos, prob.src_axis, 0.0, 10.0, prob.group_w)
    dctsn.set_source(h, 1, prob.src_pos, prob.src_axis, 20.0, 10.0, prob.group_w)
    # solve on a host-only context -> EDEVICE, dose before solve -> ESTATE
    rc = lib.dct_solve(h, None, None)
    assert rc == dctsn.DCT_EDEVICE
    out = np.zeros(ph.C)
    rc = lib.dct_dose(h, out.ctypes.data_as(ct.POINTER(ct.c_double)), 1, None, None)
    assert rc == dctsn.DCT_ESTATE
    assert "no valid solve" in dctsn.last_error(h)
    # device-buffer forms: a NULL density is rejected before any device call,
    # the adjoint needs a kept solve
    assert lib.dct_set_density_dev(h, None) == dctsn.DCT_EINVAL
    assert lib.dct_adjoint_dev(h, None, None, None, None, None, None) == dctsn.DCT_ESTATE


def test_null_context():
    lib = dctsn.lib()
    assert lib.dct_set_geometry(None, 1, 1, 1, 1.0, 1.0, 1.0, None, None, None) == dctsn.DCT_EINVAL
    assert lib.dct_destroy(None) == dctsn.DCT_OK


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of dct_opts and dct_stats have the header's field
    offsets and sizes (a field added on one side only would shift the rest)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"dct_opts": dctsn.dct_opts, "dct_stats": dctsn.dct_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dctsn.h"', "int main(void) {"]
    for name, py in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, py in structs.items():
        assert got[(name, "size")] == ct.sizeof(py), name
        for fname, _ in py._fields_:
            assert got[(name, fname)] == getattr(py, fname).offset, (name, fname)
