"""FP64 CPU oracle for the discrete-ordinates CT dose method (arXiv:1811.12391).

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline load this module; the product library never does, and the two share
no code.  The arithmetic lives in ``dct_oracle.c`` (plain C loops, FP64); this
file only builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over directions / voxels only;
    each cell's arithmetic is in a fixed order, so thread count does not change
    results)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ct.CDLL(_LIB)
        _declare(_lib)
    return _lib


_d = ct.POINTER(ct.c_double)
_i = ct.POINTER(ct.c_int)
_u8 = ct.POINTER(ct.c_uint8)
_l = ct.POINTER(ct.c_long)


def _declare(L):
    L.orc_real_sh.argtypes = [ct.c_int, ct.c_double, ct.c_double, ct.c_double, _d]
    L.orc_real_sh.restype = ct.c_int
    L.orc_moment_maps.argtypes = [ct.c_int, ct.c_int, _d, _d, _d, _d]
    L.orc_moment_maps.restype = ct.c_int
    L.orc_siddon.argtypes = [ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _d, _d, ct.c_int, _i, _d]
    L.orc_siddon.restype = ct.c_int
    L.orc_uncollided.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d, ct.c_int, ct.c_int, _d,
                                 ct.c_int, _d, _d, ct.c_double, ct.c_double, _d, ct.c_int, _d])
    L.orc_uncollided.restype = ct.c_int
    L.orc_dd_cell.argtypes = [ct.c_double, ct.c_double, _d, _d, ct.c_int, _d, _d]
    L.orc_dd_cell.restype = ct.c_int
    L.orc_sweep.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, ct.c_int, _d, _d, _d, ct.c_int,
                            ct.c_int, _d, _d])
    L.orc_sweep.restype = ct.c_long
    L.orc_sweep2.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, ct.c_int, _d, _d, _d, ct.c_int,
                             ct.c_int, _d, _d, _u8, _u8])
    L.orc_sweep2.restype = ct.c_long
    L.orc_sweep_adjoint.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, ct.c_int, _d, _d, _u8, ct.c_int, _d])
    L.orc_sweep_adjoint.restype = ct.c_int
    L.orc_adjoint.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d,
                              ct.c_int, ct.c_int, ct.c_int, _d, _d, _d,
                              ct.c_int, _d, _d,
                              ct.c_int, _d, _d, ct.c_double, ct.c_double, _d, _d,
                              ct.c_double, ct.c_int, _i, _i, ct.c_int, ct.c_int,
                              _d, _d, _d, _i])
    L.orc_adjoint.restype = ct.c_int
    L.orc_first_collision.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d, ct.c_int, ct.c_int, _d,
                                      _d, _d, _d, ct.c_int, _d])
    L.orc_first_collision.restype = ct.c_int
    L.orc_solve.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d,
                            ct.c_int, ct.c_int, ct.c_int, _d, _d, _d,
                            ct.c_int, _d, _d,
                            ct.c_int, _d, _d, ct.c_double, ct.c_double, _d, _d,
                            ct.c_double, ct.c_int, _i, ct.c_int, _d, ct.c_int,
                            _d, _d, _d, _i, _d, _d, _l])
    L.orc_solve.restype = ct.c_int
    L.orc_solve_sup.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d,
                                ct.c_int, ct.c_int, ct.c_int, _d, _d, _d,
                                ct.c_int, _d, _d,
                                ct.c_int, ct.c_int, _d, _d, ct.c_double, ct.c_double, _d, _d,
                                ct.c_double, ct.c_int, _i, ct.c_int, _d, ct.c_int,
                                _d, _d, _d, _i, _d, _d, _l])
    L.orc_solve_sup.restype = ct.c_int
    L.orc_scatter_moments.argtypes = [ct.c_long, _u8, _d, ct.c_int, ct.c_int, _d, ct.c_int, ct.c_int, _d, _d, _d,
                                      ct.c_int]
    L.orc_scatter_moments.restype = ct.c_int
    L.orc_solve_fixed.argtypes = ([ct.c_int] * 3 + [ct.c_double] * 3 + [_d, _u8, _d,
                                  ct.c_int, ct.c_int, ct.c_int, _d, _d, _d,
                                  ct.c_int, _d, _d, _d, _d,
                                  ct.c_double, ct.c_int, ct.c_int, ct.c_int,
                                  _d, _d, _i, _d, _d])
    L.orc_solve_fixed.restype = ct.c_int


def _p(a, t=_d):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except Exception:
        return 1


def real_sh(L: int, omega) -> np.ndarray:
    Y = np.zeros((L + 1) ** 2)
    rc = lib().orc_real_sh(L, float(omega[0]), float(omega[1]), float(omega[2]), _p(Y))
    assert rc == 0
    return Y


def moment_maps(L: int, dirs, w):
    dirs, w = _f64(dirs), _f64(w)
    N, Nm = dirs.shape[0], (L + 1) ** 2
    M = np.zeros((N, Nm))
    D = np.zeros((Nm, N))
    assert lib().orc_moment_maps(L, N, _p(dirs), _p(w), _p(M), _p(D)) == 0
    return M, D


def scatter_moments(material, density, sigma_s, L, gf, gt, phi, base=None, threads=None):
    """Scattering source moments of eq. (2) that the flux moments phi[Nm][C]
    of group gf put into group gt: base + rho s_l^{gf->gt}[m] phi (per moment
    of degree l).  sigma_s is [M][>=L+1][G][G] (from, to)."""
    ss = _f64(sigma_s[:, : L + 1])
    G = ss.shape[-1]
    mat = np.ascontiguousarray(material, dtype=np.uint8)
    rho, phi = _f64(density), _f64(phi)
    C = mat.shape[0]
    out = np.zeros(((L + 1) ** 2, C))
    b = None if base is None else _f64(base)
    rc = lib().orc_scatter_moments(C, _p(mat, _u8), _p(rho), G, L, _p(ss), int(gf), int(gt), _p(phi), _p(b), _p(out),
                                   threads or default_threads())
    assert rc == 0
    return out


def solve_fixed(ph, xs, dirs, w, L, ext, inflow_dir=None, *, tol=1e-6, max_iter=1000, fixup=True, threads=None):
    """Collided solve of one right-hand side from a given fixed source
    ext[G][Nm][C] (any moments) with the angular inflow inflow_dir[G][N] on
    every boundary face (None: vacuum).  Returns (phi[G][Nm][C], dose[C],
    iters[G], eps[G], bal[G][3])."""
    G, M = xs.sigma_t.shape[1], xs.sigma_t.shape[0]
    st, ss, ka = _f64(xs.sigma_t), _f64(xs.sigma_s[:, : L + 1]), _f64(xs.kerma)
    dirs, w = _f64(dirs), _f64(w)
    N, Nm, C = dirs.shape[0], (L + 1) ** 2, ph.C
    ext = _f64(ext).reshape(G, Nm, C)
    ind = None if inflow_dir is None else _f64(inflow_dir).reshape(G, N)
    mat = np.ascontiguousarray(ph.material, dtype=np.uint8)
    rho, org = _f64(ph.density), _f64(ph.origin)
    phi = np.zeros((G, Nm, C))
    dose = np.zeros(C)
    iters = np.zeros(G, dtype=np.int32)
    eps = np.zeros(G)
    bal = np.zeros((G, 3))
    rc = lib().orc_solve_fixed(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, _p(org), _p(mat, _u8), _p(rho),
                               G, M, L, _p(st), _p(ss), _p(ka), N, _p(dirs), _p(w), _p(ext), _p(ind),
                               float(tol), int(max_iter), int(fixup), threads or default_threads(),
                               _p(phi), _p(dose), _p(iters, _i), _p(eps), _p(bal))
    if rc != 0:
        raise RuntimeError("oracle fixed-source solve failed: %d" % rc)
    return phi, dose, iters, eps, bal


def siddon(grid, p, x):
    nx, ny, nz, dx, dy, dz, org = grid
    cap = nx + ny + nz + 8
    vox = np.zeros(cap, dtype=np.int32)
    ln = np.zeros(cap)
    org, p, x = _f64(org), _f64(p), _f64(x)
    ns = lib().orc_siddon(nx, ny, nz, dx, dy, dz, _p(org), _p(p), _p(x), cap, _p(vox, _i), _p(ln))
    assert ns >= 0
    return vox[:ns].copy(), ln[:ns].copy()


def dd_cell(q, sig, c, pin, fixup=True):
    c, pin = _f64(c), _f64(pin)
    pc = np.zeros(1)
    pout = np.zeros(3)
    nf = lib().orc_dd_cell(float(q), float(sig), _p(c), _p(pin), int(fixup), _p(pc), _p(pout))
    return float(pc[0]), pout, nf


def sweep(shape, spacing, sigt, dirs, q, inflow=None, fixup=True, threads=None):
    nx, ny, nz = shape
    dx, dy, dz = spacing
    sigt, dirs, q = _f64(sigt), _f64(dirs), _f64(q)
    N = dirs.shape[0]
    psi = np.zeros((N, nx * ny * nz))
    leak = np.zeros((N, 3))
    infl = None if inflow is None else _f64(np.broadcast_to(inflow, (N,)))
    nf = lib().orc_sweep(nx, ny, nz, dx, dy, dz, _p(sigt), N, _p(dirs), _p(q), _p(infl), int(fixup),
                         threads or default_threads(), _p(psi), _p(leak))
    return psi, leak, nf


def sweep_masked(shape, spacing, sigt, dirs, q, fixup=True, mask_in=None, threads=None):
    """Sweep with vacuum inflow returning (psi, mask): the fixed-face set of
    every cell (bits x=1, y=2, z=4); with mask_in the fixup is frozen to it."""
    nx, ny, nz = shape
    dx, dy, dz = spacing
    sigt, dirs, q = _f64(sigt), _f64(dirs), _f64(q)
    N = dirs.shape[0]
    psi = np.zeros((N, nx * ny * nz))
    mask = np.zeros((N, nx * ny * nz), dtype=np.uint8)
    mi = None if mask_in is None else np.ascontiguousarray(mask_in, dtype=np.uint8)
    lib().orc_sweep2(nx, ny, nz, dx, dy, dz, _p(sigt), N, _p(dirs), _p(q), None, int(fixup),
                     threads or default_threads(), _p(psi), None, _p(mi, _u8), _p(mask, _u8) if mi is None else None)
    return psi, (mask if mi is None else mi)


def sweep_adjoint(shape, spacing, sigt, dirs, s, mask, threads=None):
    """Transpose of the frozen-mask sweep: weights on psi -> weights on q."""
    nx, ny, nz = shape
    dx, dy, dz = spacing
    sigt, dirs, s = _f64(sigt), _f64(dirs), _f64(s)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    lam = np.zeros_like(s)
    lib().orc_sweep_adjoint(nx, ny, nz, dx, dy, dz, _p(sigt), dirs.shape[0], _p(dirs), _p(s), _p(mask, _u8),
                            threads or default_threads(), _p(lam))
    return lam


@dataclass
class AdjointResult:
    R: float               # sum_b sum_v roi_v dose_b(v)
    d_density: np.ndarray  # [C]
    d_group_w: np.ndarray  # [G]
    iters_adj: np.ndarray  # [B][G]


def adjoint(ph, xs, dirs, w, L, pos, axis, fan_deg, cone_deg, group_w, roi, *, tol=1e-6, max_iter=1000,
            fixed_iters=None, fixed_iters_adj=None, fixup=True, threads=None) -> AdjointResult:
    G, M = xs.sigma_t.shape[1], xs.sigma_t.shape[0]
    st, ss, ka = _f64(xs.sigma_t), _f64(xs.sigma_s[:, : L + 1]), _f64(xs.kerma)
    dirs, w = _f64(dirs), _f64(w)
    pos, axis = _f64(pos).reshape(-1, 3), _f64(axis).reshape(-1, 3)
    B = pos.shape[0]
    mat = np.ascontiguousarray(ph.material, dtype=np.uint8)
    rho, org, gw, roi = _f64(ph.density), _f64(ph.origin), _f64(group_w), _f64(roi)
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, dtype=np.int32)
    fa = None if fixed_iters_adj is None else np.ascontiguousarray(fixed_iters_adj, dtype=np.int32)
    R = np.zeros(1)
    dr = np.zeros(ph.C)
    dg = np.zeros(G)
    ia = np.zeros((B, G), dtype=np.int32)
    rc = lib().orc_adjoint(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, _p(org), _p(mat, _u8), _p(rho),
                           G, M, L, _p(st), _p(ss), _p(ka), dirs.shape[0], _p(dirs), _p(w),
                           B, _p(pos), _p(axis), float(fan_deg), float(cone_deg), _p(gw), _p(roi),
                           float(tol), int(max_iter), _p(fi, _i), _p(fa, _i), int(fixup), threads or default_threads(),
                           _p(R), _p(dr), _p(dg), _p(ia, _i))
    if rc != 0:
        raise RuntimeError("oracle adjoint failed: %d" % rc)
    return AdjointResult(float(R[0]), dr, dg, ia)


def adjoint_problem(prob, roi, **kw) -> AdjointResult:
    return adjoint(prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis,
                   prob.fan_deg, prob.cone_deg, prob.group_w, roi, **kw)


def uncollided(ph, xs_sigma_t, pos, axis, fan_deg, cone_deg, group_w, threads=None):
    pos, axis, gw = _f64(pos).reshape(-1, 3), _f64(axis).reshape(-1, 3), _f64(group_w)
    st = _f64(xs_sigma_t)
    M, G = st.shape
    B = pos.shape[0]
    out = np.zeros((B, G, ph.C))
    mat = np.ascontiguousarray(ph.material, dtype=np.uint8)
    rho = _f64(ph.density)
    org = _f64(ph.origin)
    lib().orc_uncollided(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, _p(org), _p(mat, _u8), _p(rho), G, M,
                         _p(st), B, _p(pos), _p(axis), float(fan_deg), float(cone_deg), _p(gw),
                         threads or default_threads(), _p(out))
    return out


def first_collision(ph, sigma_s, L, p, phi_u_b, ext_iso=None, threads=None):
    """ext[G][Nm][C] of one right-hand side from its uncollided flux [G][C]."""
    ss = _f64(sigma_s[:, : L + 1])
    G = ss.shape[-1]
    Nm = (L + 1) ** 2
    ext = np.zeros((G, Nm, ph.C))
    mat = np.ascontiguousarray(ph.material, dtype=np.uint8)
    rho, org, p, pu = _f64(ph.density), _f64(ph.origin), _f64(p), _f64(phi_u_b)
    ei = None if ext_iso is None else _f64(ext_iso)
    lib().orc_first_collision(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, _p(org), _p(mat, _u8), _p(rho), G, L,
                              _p(ss), _p(p), _p(pu), _p(ei), threads or default_threads(), _p(ext))
    return ext


@dataclass
class OracleResult:
    phi_u: np.ndarray      # [B][G][C]
    phi: np.ndarray        # [B][G][Nm][C] collided moments
    dose: np.ndarray       # [B][C]
    iters: np.ndarray      # [B][G]
    eps: np.ndarray        # [B][G]
    balance: np.ndarray    # [B][G][3] production, removal, leakage
    nfix: int


def solve(ph, xs, dirs, w, L, pos, axis, fan_deg, cone_deg, group_w, *, ext_iso=None, tol=1e-6,
          max_iter=1000, fixed_iters=None, fixup=True, test_inflow=None, threads=None,
          B_subset=None, superpose=1) -> OracleResult:
    """Full FP64 solve; ``xs`` needs sigma_t [M][G], sigma_s [M][L+1][G][G]
    (only l <= L used), kerma [M][G].  With ``superpose`` = S > 1 every S
    consecutive sources form one right-hand side (one collided solve of
    their summed first-collision source; the outputs are per right-hand
    side, phi_u summed over its sources)."""
    G = xs.sigma_t.shape[1]
    M = xs.sigma_t.shape[0]
    st = _f64(xs.sigma_t)
    ss = _f64(xs.sigma_s[:, : L + 1])
    ka = _f64(xs.kerma)
    dirs, w = _f64(dirs), _f64(w)
    N = dirs.shape[0]
    pos, axis = _f64(pos).reshape(-1, 3), _f64(axis).reshape(-1, 3)
    B = pos.shape[0]
    S = int(superpose)
    if S < 1 or B % S:
        raise ValueError(f"superpose={S} must divide the number of sources {B}")
    R = B // S
    C = ph.C
    Nm = (L + 1) ** 2
    phi_u = np.zeros((R, G, C))
    phi = np.zeros((R, G, Nm, C))
    dose = np.zeros((R, C))
    iters = np.zeros((R, G), dtype=np.int32)
    eps = np.zeros((R, G))
    bal = np.zeros((R, G, 3))
    nfix = ct.c_long(0)
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, dtype=np.int32)
    ei = None if ext_iso is None else _f64(ext_iso).reshape(G, C)
    ti = None if test_inflow is None else _f64(test_inflow).reshape(G)
    mat = np.ascontiguousarray(ph.material, dtype=np.uint8)
    rho = _f64(ph.density)
    org = _f64(ph.origin)
    gw = _f64(group_w)
    rc = lib().orc_solve_sup(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, _p(org), _p(mat, _u8), _p(rho),
                         G, M, L, _p(st), _p(ss), _p(ka), N, _p(dirs), _p(w),
                         B, S, _p(pos), _p(axis), float(fan_deg), float(cone_deg), _p(gw), _p(ei),
                         float(tol), int(max_iter), _p(fi, _i), int(fixup), _p(ti),
                         threads or default_threads(),
                         _p(phi_u), _p(phi), _p(dose), _p(iters, _i), _p(eps), _p(bal), ct.byref(nfix))
    if rc != 0:
        raise RuntimeError("oracle solve failed: %d" % rc)
    return OracleResult(phi_u, phi, dose, iters, eps, bal, int(nfix.value))


def solve_problem(prob, **kw) -> OracleResult:
    return solve(prob.phantom, prob.xs, prob.dirs, prob.weights, prob.L, prob.src_pos, prob.src_axis,
                 prob.fan_deg, prob.cone_deg, prob.group_w, **kw)


def effective_dose(res, phantom, edges_keV, energy_keV, factor, zero_material=None, summed=False):
    """Fluence-to-dose conversion (Sec. III-A, dose comparison paragraph):
    group-wise conversion factors taken from a table by linear interpolation
    at each group's mid energy (the end value beyond either end of the
    table), applied to the total (uncollided + collided) scalar fluence of
    every group; voxels of flagged materials (air) get zero dose.  ``res`` is
    an OracleResult; group g = 0 is the highest energy (edges descending)."""
    edges = np.asarray(edges_keV, dtype=np.float64)
    mid = 0.5 * (edges[:-1] + edges[1:])
    h = np.interp(mid, np.asarray(energy_keV, dtype=np.float64), np.asarray(factor, dtype=np.float64))
    total = res.phi_u + res.phi[:, :, 0]                     # [B][G][C]
    out = np.zeros((total.shape[0], total.shape[2]))
    for g in range(total.shape[1]):                          # group order, as the dose tally
        out += h[g] * total[:, g]
    if zero_material is not None:
        out[:, np.asarray(zero_material, dtype=bool)[phantom.material]] = 0.0
    return out.sum(axis=0) if summed else out
