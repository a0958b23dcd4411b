"""Python binding of the dctsn C ABI (include/dctsn.h): argument marshalling only.

Every step of the solve runs in the HIP library ``libdctsn.so``; this module
converts numpy arrays / torch tensors to pointers and status codes to
exceptions.  If the library is not built, loading fails loudly: there is no
Python or CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdctsn.so")

DCT_OK, DCT_EINVAL, DCT_ESTATE, DCT_EDEVICE, DCT_ENOMEM, DCT_ENOTCONV, DCT_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
DCT_FP64, DCT_FP32, DCT_FP32_BF16MAP, DCT_FP32_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": DCT_FP64, "fp32": DCT_FP32, "fp32_bf16map": DCT_FP32_BF16MAP, "fp32_bf16x3": DCT_FP32_BF16X3}
STATUS_NAMES = {0: "DCT_OK", -1: "DCT_EINVAL", -2: "DCT_ESTATE", -3: "DCT_EDEVICE", -4: "DCT_ENOMEM",
                -5: "DCT_ENOTCONV", -6: "DCT_ENUMERIC"}

# every symbol include/dctsn.h declares
EXPORTS = ["dct_create", "dct_destroy", "dct_last_error", "dct_set_geometry", "dct_set_xs",
           "dct_set_quadrature", "dct_set_source", "dct_set_volume_source", "dct_solve", "dct_dose",
           "dct_dose_dev", "dct_effective_dose", "dct_effective_dose_noalloc", "dct_adjoint", "dct_moments",
           "dct_roi_dose", "dct_set_density_dev", "dct_adjoint_dev"]


class DctError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class dct_opts(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("tol", ct.c_double), ("max_iter", ct.c_int),
                ("fixed_iters", ct.POINTER(ct.c_int)), ("fixup", ct.c_int),
                ("test_inflow", ct.POINTER(ct.c_double)), ("chunk", ct.c_int), ("use_graph", ct.c_int),
                ("profile", ct.c_int), ("keep_adjoint", ct.c_int), ("autotune", ct.c_int),
                ("sweep_bk", ct.c_int), ("sweep_sync", ct.c_int), ("superpose", ct.c_int),
                ("stall_window", ct.c_int), ("sweep_chain", ct.c_int), ("fuse_maps", ct.c_int),
                ("warm_start", ct.c_int), ("accel_depth", ct.c_int), ("sweep_rhs_chain", ct.c_int),
                ("rhs_streams", ct.c_int)]


class dct_stats(ct.Structure):
    _fields_ = [("iters", ct.POINTER(ct.c_int)), ("eps", ct.POINTER(ct.c_double)),
                ("balance", ct.POINTER(ct.c_double)), ("sweep_updates", ct.c_longlong),
                ("sweep_launches", ct.c_int), ("sweep_ms", ct.c_double), ("solve_ms", ct.c_double),
                ("iteration_sets", ct.c_int), ("sweep_bk", ct.c_int), ("sweep_sync", ct.c_int),
                ("tune_ms", ct.c_double), ("sweep_launches_all", ct.c_longlong), ("sweep_chain", ct.c_int),
                ("fused_maps", ct.c_int), ("warm_start", ct.c_int), ("fused_ms", ct.c_double),
                ("fused_launches", ct.c_int), ("sweep_rhs_chain", ct.c_int), ("rhs_streams", ct.c_int)]


_lib = None
_d = ct.POINTER(ct.c_double)
_u8 = ct.POINTER(ct.c_uint8)
_vp = ct.c_void_p


def lib():
    """Load libdctsn.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"dctsn HIP library not built: {LIB_PATH} missing "
                               "(run __graft_entry__.build() or python paper_1811_12391_amd/build.py)")
        L = ct.CDLL(LIB_PATH)
        L.dct_create.argtypes = [ct.POINTER(_vp), ct.c_int, _vp]
        L.dct_destroy.argtypes = [_vp]
        L.dct_last_error.argtypes = [_vp]
        L.dct_last_error.restype = ct.c_char_p
        L.dct_set_geometry.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_double,
                                       _d, _u8, _d]
        L.dct_set_xs.argtypes = [_vp, ct.c_int, _d, ct.c_int, ct.c_int, _d, _d, _d]
        L.dct_set_quadrature.argtypes = [_vp, ct.c_int, _d, _d]
        L.dct_set_source.argtypes = [_vp, ct.c_int, _d, _d, ct.c_double, ct.c_double, _d]
        L.dct_set_volume_source.argtypes = [_vp, _d]
        L.dct_solve.argtypes = [_vp, ct.POINTER(dct_opts), ct.POINTER(dct_stats)]
        L.dct_dose.argtypes = [_vp, _d, ct.c_int, _d, _d]
        L.dct_dose_dev.argtypes = [_vp, _vp, ct.c_int, _vp, _vp]
        L.dct_roi_dose.argtypes = [_vp, _d, _d]
        L.dct_adjoint.argtypes = [_vp, _d, ct.POINTER(dct_opts), _d, _d, _d, ct.POINTER(dct_stats)]
        L.dct_adjoint_dev.argtypes = [_vp, _vp, ct.POINTER(dct_opts), _d, _vp, _vp, ct.POINTER(dct_stats)]
        L.dct_set_density_dev.argtypes = [_vp, _vp]
        L.dct_moments.argtypes = [_vp, _d]
        L.dct_effective_dose.argtypes = [_vp, ct.c_int, _d, _d, _u8, _d, ct.c_int]
        L.dct_effective_dose_noalloc.argtypes = [_vp, ct.c_int, _d, _d, _u8, _vp, ct.c_int]
        for n in EXPORTS:
            if n != "dct_last_error":
                getattr(L, n).restype = ct.c_int
        _lib = L
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_d):
    return None if a is None else a.ctypes.data_as(t)


def _dev_ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr())


def _dev_f64(t, n, what):
    """Device pointer of a contiguous float64 GPU tensor of n elements (or None),
    after the work queued on torch's current stream has finished."""
    if t is None:
        return None
    import torch

    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what}: expected a contiguous float64 GPU tensor of {n} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    torch.cuda.current_stream(t.device).synchronize()
    return ct.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C-named calls
def create(device: int = 0, stream=None):
    h = _vp()
    rc = lib().dct_create(ct.byref(h), int(device), stream)
    if rc != DCT_OK:
        raise DctError(rc, lib().dct_last_error(None).decode())
    return h


def destroy(h):
    lib().dct_destroy(h)


def last_error(h) -> str:
    return lib().dct_last_error(h).decode()


def _chk(h, rc, ok=(DCT_OK,)):
    if rc not in ok:
        raise DctError(rc, last_error(h))
    return rc


def set_geometry(h, nx, ny, nz, dx, dy, dz, origin, material, density):
    origin, density = _f64(origin), _f64(density)
    material = np.ascontiguousarray(material, dtype=np.uint8)
    return _chk(h, lib().dct_set_geometry(h, nx, ny, nz, dx, dy, dz, _p(origin), _p(material, _u8), _p(density)))


def set_xs(h, G, edges, M, L, sigma_t, sigma_s, kerma):
    edges, sigma_t, sigma_s, kerma = _f64(edges), _f64(sigma_t), _f64(sigma_s), _f64(kerma)
    return _chk(h, lib().dct_set_xs(h, G, _p(edges), M, L, _p(sigma_t), _p(sigma_s), _p(kerma)))


def set_quadrature(h, n, dirs, w):
    dirs, w = _f64(dirs), _f64(w)
    return _chk(h, lib().dct_set_quadrature(h, n, _p(dirs), _p(w)))


def set_source(h, B, pos, axis, fan_deg, cone_deg, group_w):
    pos, axis, group_w = _f64(pos), _f64(axis), _f64(group_w)
    return _chk(h, lib().dct_set_source(h, B, _p(pos), _p(axis), fan_deg, cone_deg, _p(group_w)))


def set_volume_source(h, S):
    S = _f64(S)
    return _chk(h, lib().dct_set_volume_source(h, _p(S)))


@dataclass
class SolveStats:
    status: int
    iters: np.ndarray
    eps: np.ndarray
    balance: np.ndarray
    sweep_updates: int
    sweep_launches: int
    sweep_ms: float
    solve_ms: float
    iteration_sets: int
    sweep_bk: int
    sweep_sync: int
    tune_ms: float
    sweep_launches_all: int = 0
    sweep_chain: int = 1
    fused_maps: int = 0
    warm_start: int = 0
    fused_ms: float = 0.0
    fused_launches: int = 0
    sweep_rhs_chain: int = 1
    rhs_streams: int = 1


def solve(h, B, G, *, precision="fp64", tol=1e-6, max_iter=1000, fixed_iters=None, fixup=True,
          test_inflow=None, chunk=0, use_graph=False, profile=False, keep_adjoint=False, autotune=False,
          sweep_bk=0, sweep_sync=0, superpose=1, stall_window=0, sweep_chain=0, fuse_maps=0,
          warm_start=False, accel_depth=0, sweep_rhs_chain=0, rhs_streams=0, allow_notconv=False) -> SolveStats:
    """B = number of sources; with superpose = S > 1 the per-right-hand-side
    outputs have B // S rows."""
    o = dct_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.tol = tol
    o.max_iter = max_iter
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, dtype=np.int32)
    ti = _f64(test_inflow)
    o.fixed_iters = _p(fi, ct.POINTER(ct.c_int)) if fi is not None else None
    o.fixup = int(fixup)
    o.test_inflow = _p(ti) if ti is not None else None
    o.chunk = int(chunk)
    o.use_graph = int(use_graph)
    o.profile = int(profile)
    o.keep_adjoint = int(keep_adjoint)
    o.autotune = int(autotune)
    o.sweep_bk = int(sweep_bk)
    o.sweep_sync = int(sweep_sync)
    o.superpose = int(superpose)
    o.stall_window = int(stall_window)
    o.sweep_chain = int(sweep_chain)
    o.fuse_maps = int(fuse_maps)
    o.warm_start = int(warm_start)
    o.accel_depth = int(accel_depth)
    o.sweep_rhs_chain = int(sweep_rhs_chain)
    o.rhs_streams = int(rhs_streams)
    S = max(1, int(superpose))
    if B % S:
        raise ValueError(f"superpose={S} must divide the number of sources {B}")
    B = B // S
    iters = np.zeros((B, G), dtype=np.int32)
    eps = np.zeros((B, G))
    bal = np.zeros((B, G, 3))
    st = dct_stats()
    st.iters = iters.ctypes.data_as(ct.POINTER(ct.c_int))
    st.eps = _p(eps)
    st.balance = _p(bal)
    ok = (DCT_OK, DCT_ENOTCONV) if allow_notconv else (DCT_OK,)
    rc = _chk(h, lib().dct_solve(h, ct.byref(o), ct.byref(st)), ok)
    return SolveStats(rc, iters, eps, bal, st.sweep_updates, st.sweep_launches, st.sweep_ms, st.solve_ms,
                      st.iteration_sets, st.sweep_bk, st.sweep_sync, st.tune_ms, st.sweep_launches_all,
                      st.sweep_chain, st.fused_maps, st.warm_start, st.fused_ms, st.fused_launches,
                      st.sweep_rhs_chain, st.rhs_streams)


def dose(h, B, G, C, *, summed=False, want_phi=False):
    out = np.zeros(C if summed else (B, C))
    pu = np.zeros((B, G, C)) if want_phi else None
    pc = np.zeros((B, G, C)) if want_phi else None
    _chk(h, lib().dct_dose(h, _p(out), int(summed), _p(pu), _p(pc)))
    return (out, pu, pc) if want_phi else out


def effective_dose(h, B, C, energy_keV, factor, *, zero_material=None, summed=False):
    """Fluence-to-dose conversion of the last solve: per-group factors from a
    table (linear in energy at each group's mid energy, flat beyond the
    ends), zero in the flagged materials; B = right-hand sides."""
    e, f = _f64(energy_keV).reshape(-1), _f64(factor).reshape(-1)
    if e.size != f.size:
        raise ValueError("energy and factor tables differ in length")
    z = None if zero_material is None else np.ascontiguousarray(zero_material, dtype=np.uint8)
    out = np.zeros(C if summed else (B, C))
    _chk(h, lib().dct_effective_dose(h, int(e.size), _p(e), _p(f), _p(z, _u8), _p(out), int(summed)))
    return out


def effective_dose_noalloc(h, energy_keV, factor, out_t, *, zero_material=None, summed=False):
    """As effective_dose, into a float64 torch tensor on the context's device,
    through the entry point that allocates no device memory."""
    e, f = _f64(energy_keV).reshape(-1), _f64(factor).reshape(-1)
    if e.size != f.size:
        raise ValueError("energy and factor tables differ in length")
    z = None if zero_material is None else np.ascontiguousarray(zero_material, dtype=np.uint8)
    return _chk(h, lib().dct_effective_dose_noalloc(h, int(e.size), _p(e), _p(f), _p(z, _u8), _dev_ptr(out_t),
                                                    int(summed)))


def dose_dev(h, dose_t, summed=False, phi_u_t=None, phi_c_t=None):
    """Write results into device tensors (float64 torch tensors on the context's device)."""
    return _chk(h, lib().dct_dose_dev(h, _dev_ptr(dose_t), int(summed), _dev_ptr(phi_u_t), _dev_ptr(phi_c_t)))


def roi_dose(h, C, roi) -> float:
    """R = sum_b sum_v roi[v] dose_b(v) of the last solve, reduced on the device."""
    roi = _f64(roi).reshape(-1)
    if roi.size != C:
        raise ValueError(f"roi has {roi.size} entries, expected {C}")
    R = np.zeros(1)
    _chk(h, lib().dct_roi_dose(h, _p(roi), _p(R)))
    return float(R[0])


@dataclass
class AdjointResult:
    R: float
    d_density: np.ndarray     # [C] (from adjoint_dev: the caller's GPU tensor)
    d_group_w: np.ndarray     # [G] (likewise)
    iters: np.ndarray         # [B][G] adjoint iterations
    eps: np.ndarray
    solve_ms: float


def adjoint(h, B, G, C, roi, *, tol=1e-6, max_iter=1000, fixed_iters=None, chunk=0,
            stall_window=0) -> AdjointResult:
    """Gradient of sum_b sum_v roi[v] dose_b(v) after a solve with keep_adjoint=True."""
    roi = _f64(roi).reshape(-1)
    if roi.size != C:
        raise ValueError(f"roi has {roi.size} entries, expected {C}")
    o = dct_opts()
    o.tol = tol
    o.max_iter = max_iter
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, dtype=np.int32)
    o.fixed_iters = _p(fi, ct.POINTER(ct.c_int)) if fi is not None else None
    o.chunk = int(chunk)
    o.stall_window = int(stall_window)
    R = np.zeros(1)
    dd = np.zeros(C)
    dg = np.zeros(G)
    iters = np.zeros((B, G), dtype=np.int32)
    eps = np.zeros((B, G))
    st = dct_stats()
    st.iters = iters.ctypes.data_as(ct.POINTER(ct.c_int))
    st.eps = _p(eps)
    _chk(h, lib().dct_adjoint(h, _p(roi), ct.byref(o), _p(R), _p(dd), _p(dg), ct.byref(st)))
    return AdjointResult(float(R[0]), dd, dg, iters, eps, st.solve_ms)


def set_density_dev(h, C, density_t):
    """New voxel densities from a float64 GPU tensor of C elements (grid and
    materials of the last set_geometry kept)."""
    return _chk(h, lib().dct_set_density_dev(h, _dev_f64(density_t, C, "density")))


def adjoint_dev(h, B, G, C, roi_t, d_density_t=None, d_group_w_t=None, *, tol=1e-6, max_iter=1000,
                fixed_iters=None, chunk=0, stall_window=0) -> AdjointResult:
    """As adjoint, with the ROI weights read from and the gradients written into
    float64 GPU tensors; d_density / d_group_w of the result are those tensors."""
    o = dct_opts()
    o.tol = tol
    o.max_iter = max_iter
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, dtype=np.int32)
    o.fixed_iters = _p(fi, ct.POINTER(ct.c_int)) if fi is not None else None
    o.chunk = int(chunk)
    o.stall_window = int(stall_window)
    R = np.zeros(1)
    iters = np.zeros((B, G), dtype=np.int32)
    eps = np.zeros((B, G))
    st = dct_stats()
    st.iters = iters.ctypes.data_as(ct.POINTER(ct.c_int))
    st.eps = _p(eps)
    _chk(h, lib().dct_adjoint_dev(h, _dev_f64(roi_t, C, "roi"), ct.byref(o), _p(R),
                                  _dev_f64(d_density_t, C, "d_density"), _dev_f64(d_group_w_t, G, "d_group_w"),
                                  ct.byref(st)))
    return AdjointResult(float(R[0]), d_density_t, d_group_w_t, iters, eps, st.solve_ms)


def moments(h, B, G, Nm, C):
    out = np.zeros((B, G, Nm, C))
    _chk(h, lib().dct_moments(h, _p(out)))
    return out


# ------------------------------------------------------------------ convenience
class Solver:
    """Owns one context loaded with a ``inputs.Problem``."""

    def __init__(self, prob, device: int = 0, stream=None):
        self.prob = prob
        self.h = create(device, stream)
        ph, xs = prob.phantom, prob.xs
        set_geometry(self.h, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material, ph.density)
        set_xs(self.h, xs.G, xs.edges, xs.M, prob.L, xs.sigma_t, xs.sigma_s[:, : prob.L + 1], xs.kerma)
        set_quadrature(self.h, prob.N, prob.dirs, prob.weights)
        set_source(self.h, prob.B, prob.src_pos, prob.src_axis, prob.fan_deg, prob.cone_deg, prob.group_w)
        self.rhs = prob.B                 # right-hand sides of the last solve

    def solve(self, **kw) -> SolveStats:
        st = solve(self.h, self.prob.B, self.prob.G, **kw)
        self.rhs = self.prob.B // max(1, int(kw.get("superpose", 1)))
        return st

    def dose(self, **kw):
        return dose(self.h, self.rhs, self.prob.G, self.prob.phantom.C, **kw)

    def effective_dose(self, energy_keV, factor, **kw):
        return effective_dose(self.h, self.rhs, self.prob.phantom.C, energy_keV, factor, **kw)

    def adjoint(self, roi, **kw) -> AdjointResult:
        return adjoint(self.h, self.prob.B, self.prob.G, self.prob.phantom.C, roi, **kw)

    def set_density(self, density):
        """Replace the voxel densities (same grid and materials): a host array,
        or a float64 GPU tensor, which the library copies on the device."""
        ph = self.prob.phantom
        if getattr(density, "is_cuda", False):
            set_density_dev(self.h, ph.C, density.reshape(-1))
        else:
            set_geometry(self.h, ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.origin, ph.material, density)

    def adjoint_dev(self, roi_t, d_density_t=None, d_group_w_t=None, **kw) -> AdjointResult:
        return adjoint_dev(self.h, self.prob.B, self.prob.G, self.prob.phantom.C, roi_t, d_density_t,
                           d_group_w_t, **kw)

    def set_group_weights(self, group_w):
        p = self.prob
        set_source(self.h, p.B, p.src_pos, p.src_axis, p.fan_deg, p.cone_deg, group_w)

    def moments(self):
        return moments(self.h, self.rhs, self.prob.G, (self.prob.L + 1) ** 2, self.prob.phantom.C)

    def close(self):
        if self.h is not None:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
