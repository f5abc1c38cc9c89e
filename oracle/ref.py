"""FP64 oracle of the induced-dipole solve (Python side).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.  It shares no code with the GPU library.

The operator is A = alpha^-1 - T, where T mu is the full Ewald field of the
induced dipoles: real-space Thole-damped pairs (C part, orc_real_mutual), a
reciprocal part and the dipole self field.  The reciprocal part is either the
direct Ewald k-sum (exact; 'ksum') or smooth PME on the same grid/order as the
GPU path ('spme').  The permanent field E_perm is built the same way from the
charges, dipoles and quadrupoles with the scaled-pair correction.

The solve (PCG with the diagonal preconditioner, paper "Optimizations
opportunities" and the benchmark settings of "Performance and Scalability
Results") is the textbook preconditioned conjugate gradient; dense Cholesky is
the exact solution of the same linear system for small cases.

Inputs are duck-typed: any object with pos, box, alpha, thole, q, dip, quad,
sc_ptr, sc_j, sc_s, cutoff, ewald_alpha, grid, order (and, for the two-set model,
sc_s_d: the direct scales of the same pairs).
"""
from __future__ import annotations

import copy
import ctypes
import math
import os

import numpy as np

COULOMB = 332.0637133      # kcal*A/(mol*e^2)
DEBYE = 4.80320            # Debye per e*A

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load (building first if needed) the oracle's C part."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.orc_thole_oml.argtypes = [ctypes.c_double] * 5 + [_dp]
        L.orc_ewald_b.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
        L.orc_real_mutual.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp,
                                      _dp, ctypes.c_int, _ip, _dp, _ip, _ip, _ip, _ip]
        L.orc_real_perm.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp,
                                    _dp, _dp, _ip, _ip, _dp, ctypes.c_int, _ip, _dp, _ip, _ip, _ip, _ip]
        L.orc_ksum_field.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp,
                                     ctypes.c_int, _ip, _dp]
        L.orc_bspline.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_bspline.restype = ctypes.c_double
        L.orc_spme_spread.argtypes = [ctypes.c_int, _dp, _dp, _ip, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_spme_gather.argtypes = [ctypes.c_int, _dp, _dp, _ip, ctypes.c_int, _dp, ctypes.c_int, _ip, _dp]
        L.orc_count_pairs.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _ip, _ip, _ip, _ip]
        L.orc_polar_grad_real.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp,
                                          _dp, _dp, _dp, _dp, _ip, _ip, _dp, ctypes.c_int, _ip, _dp,
                                          _ip, _ip, _ip, _ip]
        L.orc_spme_grad.argtypes = [ctypes.c_int, _dp, _dp, _ip, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ctypes.c_int, _ip, _dp]
        L.orc_count_pairs.restype = ctypes.c_int64
        L.orc_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _d(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _outsel(n, idx):
    if idx is None:
        return n, None, None
    keep, p = _i(idx)
    return len(keep), keep, p


def cell_bins(pos, box, rc):
    """Periodic cell grid for the partner search of the real-space loops: nc[a] = floor(L_a / rc)
    cells per axis (each at least rc wide), atoms binned by their wrapped position.  Returns the
    four arrays the C loops take (nc, cell of each atom, cell start offsets, atoms by cell), or
    None where an axis has fewer than three cells (then every atom is a candidate)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    box = np.asarray(box, dtype=np.float64)
    nc = np.floor(box / rc).astype(np.int64)
    if not np.isfinite(rc) or np.any(nc < 3):
        return None
    u = pos - box * np.floor(pos / box)
    c = np.minimum(np.floor(u / box * nc).astype(np.int64), nc - 1)
    cid = (c[:, 0] * nc[1] + c[:, 1]) * nc[2] + c[:, 2]
    order = np.argsort(cid, kind="stable")
    start = np.searchsorted(cid[order], np.arange(int(np.prod(nc)) + 1))
    return (nc.astype(np.int32), cid.astype(np.int32), start.astype(np.int32), order.astype(np.int32))


def _search_args(s, rc, search):
    """ctypes arguments of the partner search: 'cells' (when the box allows it) or 'all'."""
    if search not in ("cells", "all"):
        raise ValueError(search)
    cl = cell_bins(s.pos, s.box, rc) if (search == "cells" and np.isfinite(rc)) else None
    if cl is None:
        return (), (None, None, None, None)
    keep = tuple(np.ascontiguousarray(a) for a in cl)
    return keep, tuple(a.ctypes.data_as(_ip) for a in keep)


# ----------------------------------------------------------------------------------------------
# pair functions exposed for pins
# ----------------------------------------------------------------------------------------------

def thole_lambdas(r, alpha_i, alpha_j, a_i, a_j):
    """(lambda3, lambda5, lambda7) of the Thole damping at separation r."""
    o = (ctypes.c_double * 3)()
    lib().orc_thole_oml(r, alpha_i, alpha_j, a_i, a_j, o)
    return 1.0 - o[0], 1.0 - o[1], 1.0 - o[2]


def ewald_b(r, beta):
    o = (ctypes.c_double * 4)()
    lib().orc_ewald_b(r, beta, o)
    return np.array(o[:])


def bspline(order, x, deriv=0):
    return lib().orc_bspline(order, float(x), deriv)


def self_coeff(beta: float) -> float:
    """Ewald self field of a dipole: E_self = 4 beta^3 / (3 sqrt(pi)) * mu."""
    return 4.0 * beta ** 3 / (3.0 * math.sqrt(math.pi))


def default_kmax(beta: float, tail: float = 1e-17) -> float:
    """|k| beyond which exp(-k^2/(4 beta^2)) < tail."""
    return 2.0 * beta * math.sqrt(-math.log(tail))


# ----------------------------------------------------------------------------------------------
# field components
# ----------------------------------------------------------------------------------------------

def real_mutual(s, mu, idx=None, beta=None, rc=None, free_space=False, search="cells"):
    """Real-space (Thole-damped, Ewald-screened) field of dipoles mu at atoms idx (all if None).
    free_space: no periodic images, no cutoff, beta = 0 (bare damped dipole tensor).
    search: 'cells' (a periodic cell grid finds the partners within rc) or 'all' (every pair)."""
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _, ap = _d(s.alpha)
    _, tp = _d(s.thole)
    _, mp = _d(mu)
    if free_space:
        bp, beta, rc = None, 0.0, math.inf
    else:
        _box, bp = _d(s.box)
        beta = s.ewald_alpha if beta is None else beta
        rc = s.cutoff if rc is None else rc
    n_out, _keep, ip = _outsel(n, idx)
    out = np.zeros((n_out, 3))
    _cl, cl = _search_args(s, rc, search) if not free_space else ((), (None,) * 4)
    lib().orc_real_mutual(n, pp, bp, beta, rc, ap, tp, mp, n_out, ip, out.ctypes.data_as(_dp), *cl)
    return out


def real_perm(s, idx=None, beta=None, rc=None, free_space=False, q=True, dip=True, quad=True,
              scaled=True, search="cells"):
    """Real-space permanent field of (q, d, Theta) with the scaled-pair correction (search as in
    real_mutual)."""
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _, ap = _d(s.alpha)
    _, tp = _d(s.thole)
    _, qp = _d(s.q if q else None)
    _, dp = _d(s.dip if dip else None)
    _, Qp = _d(s.quad if quad else None)
    if scaled:
        _, sp = _i(s.sc_ptr)
        _, sjp = _i(s.sc_j if len(s.sc_j) else np.zeros(1, np.int32))
        _, ssp = _d(s.sc_s if len(s.sc_s) else np.zeros(1))
    else:
        sp = sjp = ssp = None
    if free_space:
        bp, beta, rc = None, 0.0, math.inf
    else:
        _box, bp = _d(s.box)
        beta = s.ewald_alpha if beta is None else beta
        rc = s.cutoff if rc is None else rc
    n_out, _keep, ip = _outsel(n, idx)
    out = np.zeros((n_out, 3))
    _cl, cl = _search_args(s, rc, search) if not free_space else ((), (None,) * 4)
    lib().orc_real_perm(n, pp, bp, beta, rc, ap, tp, qp, dp, Qp, sp, sjp, ssp, n_out, ip,
                        out.ctypes.data_as(_dp), *cl)
    return out


def ksum_field(s, q=None, dip=None, quad=None, idx=None, beta=None, kmax=None):
    """Reciprocal-space Ewald field (direct k-sum, tin-foil, no self term) at atoms idx."""
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _box, bp = _d(s.box)
    beta = s.ewald_alpha if beta is None else beta
    kmax = default_kmax(beta) if kmax is None else kmax
    _, qp = _d(q)
    _, dp = _d(dip)
    _, Qp = _d(quad)
    n_out, _keep, ip = _outsel(n, idx)
    out = np.zeros((n_out, 3))
    lib().orc_ksum_field(n, pp, bp, beta, kmax, qp, dp, Qp, n_out, ip, out.ctypes.data_as(_dp))
    return out


def bspline_moduli(kdim: int, order: int) -> np.ndarray:
    """|sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k / K)|^2 for m = 0..K-1.  For odd order the sum
    vanishes at m = K/2; there it is replaced by the mean of its two neighbours."""
    m = np.arange(kdim)
    mk = np.array([bspline(order, k + 1.0) for k in range(order - 1)])
    ssum = np.zeros(kdim, dtype=np.complex128)
    for k in range(order - 1):
        ssum += mk[k] * np.exp(2j * np.pi * m * k / kdim)
    mod = np.abs(ssum) ** 2
    for i in range(kdim):
        if mod[i] < 1e-14:
            mod[i] = 0.5 * (mod[(i - 1) % kdim] + mod[(i + 1) % kdim])
    return mod


def spme_influence(box, grid, beta, order) -> np.ndarray:
    """theta(m) = B(m) C(m) on the full grid, C(m) = exp(-pi^2 m^2 / beta^2) / (pi V m^2), C(0) = 0,
    B(m) = prod_a 1 / |b-spline modulus|^2 (Essmann et al. 1995)."""
    box = np.asarray(box, dtype=np.float64)
    vol = float(np.prod(box))
    ms = []
    for a in range(3):
        k = np.arange(grid[a])
        signed = np.where(k <= grid[a] // 2, k, k - grid[a])
        ms.append(signed / box[a])
    mx, my, mz = np.meshgrid(*ms, indexing='ij')
    m2 = mx ** 2 + my ** 2 + mz ** 2
    with np.errstate(divide='ignore', invalid='ignore'):
        c = np.exp(-np.pi ** 2 * m2 / beta ** 2) / (np.pi * vol * m2)
    c[0, 0, 0] = 0.0
    bm = [bspline_moduli(grid[a], order) for a in range(3)]
    denom = bm[0][:, None, None] * bm[1][None, :, None] * bm[2][None, None, :]
    return c / denom


def spme_spread(s, q=None, dip=None, quad=None, grid=None):
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _box, bp = _d(s.box)
    grid = tuple(s.grid if grid is None else grid)
    _g, gp = _i(np.asarray(grid, np.int32))
    _, qp = _d(q)
    _, dp = _d(dip)
    _, Qp = _d(quad)
    Q = np.zeros(grid)
    lib().orc_spme_spread(n, pp, bp, gp, int(s.order), qp, dp, Qp, Q.ctypes.data_as(_dp))
    return Q


def spme_potential(s, Q, grid=None, beta=None):
    """psi = unnormalised inverse DFT of theta * DFT(Q)."""
    grid = tuple(s.grid if grid is None else grid)
    beta = s.ewald_alpha if beta is None else beta
    theta = spme_influence(s.box, grid, beta, s.order)
    return np.real(np.fft.ifftn(theta * np.fft.fftn(Q))) * float(np.prod(grid))


def spme_gather(s, psi, idx=None, grid=None):
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _box, bp = _d(s.box)
    grid = tuple(s.grid if grid is None else grid)
    _g, gp = _i(np.asarray(grid, np.int32))
    _psi, psp = _d(psi)
    n_out, _keep, ip = _outsel(n, idx)
    out = np.zeros((n_out, 3))
    lib().orc_spme_gather(n, pp, bp, gp, int(s.order), psp, n_out, ip, out.ctypes.data_as(_dp))
    return out


def spme_field(s, q=None, dip=None, quad=None, idx=None, grid=None, beta=None):
    """Reciprocal-space field by smooth PME (spread -> FFT convolution -> gather), no self term."""
    Q = spme_spread(s, q, dip, quad, grid)
    psi = spme_potential(s, Q, grid, beta)
    return spme_gather(s, psi, idx, grid)


def recip_field(s, q=None, dip=None, quad=None, idx=None, recip='spme', beta=None):
    if recip == 'spme':
        return spme_field(s, q, dip, quad, idx, beta=beta)
    if recip == 'ksum':
        return ksum_field(s, q, dip, quad, idx, beta=beta)
    raise ValueError(recip)


# ----------------------------------------------------------------------------------------------
# operator, permanent field, solve
# ----------------------------------------------------------------------------------------------

def _sel(a, idx):
    return a if idx is None else a[np.asarray(idx)]


def mutual_field(s, mu, recip='spme', idx=None, beta=None):
    """T mu: real-space + reciprocal + self field of the induced dipoles (recip=None: free space)."""
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, 3)
    if recip is None:
        return real_mutual(s, mu, idx, free_space=True)
    beta = s.ewald_alpha if beta is None else beta
    e = real_mutual(s, mu, idx, beta=beta)
    e += recip_field(s, dip=mu, idx=idx, recip=recip, beta=beta)
    e += self_coeff(beta) * _sel(mu, idx)
    return e


def matvec(s, mu, recip='spme', idx=None, beta=None):
    """(alpha^-1 - T) mu at atoms idx."""
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, 3)
    return _sel(mu / np.asarray(s.alpha)[:, None], idx) - mutual_field(s, mu, recip, idx, beta)


def perm_field(s, recip='spme', idx=None, beta=None):
    """E_perm: real-space (with scaled-pair correction) + reciprocal + dipole self field."""
    if recip is None:
        return real_perm(s, idx, free_space=True)
    beta = s.ewald_alpha if beta is None else beta
    e = real_perm(s, idx, beta=beta)
    e += recip_field(s, q=s.q, dip=s.dip, quad=s.quad, idx=idx, recip=recip, beta=beta)
    e += self_coeff(beta) * _sel(np.asarray(s.dip), idx)
    return e


def with_scales(s, sc_s):
    """A shallow copy of the system whose listed pairs carry the scales sc_s instead."""
    t = copy.copy(s)
    t.sc_s = np.asarray(sc_s, dtype=np.float64)
    return t


def perm_field_dp(s, recip='spme', idx=None, beta=None):
    """(E_d, E_p) of AMOEBA's two induced-dipole sets (paper "Real space scheme": a polarization
    interaction carries three scaling kinds): the permanent field with the direct scales
    s.sc_s_d (the p-scales when the system has none) and with the p-scales s.sc_s.  Each is
    perm_field of the system with that scale array."""
    sd = getattr(s, 'sc_s_d', None)
    e_p = perm_field(s, recip, idx, beta)
    e_d = e_p.copy() if sd is None else perm_field(with_scales(s, sd), recip, idx, beta)
    return e_d, e_p


def e_pol_dp(mu_d, e_p) -> float:
    """Two-set polarization energy -1/2 C sum_i mu_d,i . E_p,i in kcal/mol."""
    return e_pol(mu_d, e_p)


def rms_debye(v) -> float:
    v = np.asarray(v).reshape(-1, 3)
    return DEBYE * math.sqrt(float(np.sum(v * v)) / v.shape[0])


def e_pol(mu, e_perm) -> float:
    """Polarization energy -1/2 C sum_i mu_i . E_perm,i in kcal/mol."""
    return -0.5 * COULOMB * float(np.sum(np.asarray(mu) * np.asarray(e_perm)))


def pcg(s, rhs, recip='spme', tol_debye=1e-8, mu0=None, max_iter=1000, op=None, on_iterate=None):
    """Preconditioned CG on (alpha^-1 - T) mu = rhs with the diagonal preconditioner z = alpha r.
    Stops when the rms of z (in Debye) drops below tol_debye.  Returns (mu, iterations, history),
    iterations = number of operator applications after the initial residual.  on_iterate(k, mu,
    rms_z), if given, observes every iterate (k = 0 for the start); it changes nothing."""
    alpha = np.asarray(s.alpha, dtype=np.float64)[:, None]
    apply = op if op is not None else (lambda v: matvec(s, v, recip))
    rhs = np.asarray(rhs, dtype=np.float64).reshape(-1, 3)
    mu = np.zeros_like(rhs) if mu0 is None else np.array(mu0, dtype=np.float64).reshape(-1, 3)
    r = rhs - apply(mu) if mu0 is not None else rhs.copy()
    z = alpha * r
    hist = [rms_debye(z)]
    if on_iterate is not None:
        on_iterate(0, mu, hist[-1])
    if hist[-1] < tol_debye:
        return mu, 0, hist
    p = z.copy()
    rz = float(np.sum(r * z))
    for it in range(1, max_iter + 1):
        q = apply(p)
        gamma = rz / float(np.sum(p * q))
        mu += gamma * p
        r -= gamma * q
        z = alpha * r
        hist.append(rms_debye(z))
        if on_iterate is not None:
            on_iterate(it, mu, hist[-1])
        if hist[-1] < tol_debye:
            return mu, it, hist
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return mu, max_iter, hist


def dense_operator(s, recip='spme'):
    """The 3N x 3N matrix of (alpha^-1 - T), column by column (small systems only)."""
    n = len(s.alpha)
    a = np.zeros((3 * n, 3 * n))
    for c in range(3 * n):
        e = np.zeros(3 * n)
        e[c] = 1.0
        a[:, c] = matvec(s, e.reshape(-1, 3), recip).ravel()
    return a


def count_pairs(s, rc=None, search="cells") -> int:
    """Unordered pairs with 0 < |r| < rc under the minimum image."""
    pos, pp = _d(s.pos)
    _box, bp = _d(s.box)
    rc = s.cutoff if rc is None else rc
    _cl, cl = _search_args(s, rc, search)
    return int(lib().orc_count_pairs(pos.shape[0], pp, bp, rc, *cl))


# ----------------------------------------------------------------------------------------------
# polarization energy gradient (forces = -gradient)
# ----------------------------------------------------------------------------------------------

def polar_gradient(s, mu, recip='spme', idx=None, search="cells"):
    """dE_pol/dr (kcal/mol/A) at the converged dipoles mu (E_pol stationary in mu): the real-space
    pair terms (mutual, permanent with the scaled-pair correction) and, with recip='spme', the
    smooth-PME terms; recip=None is free space (no images, no cutoff, beta = 0).  The dipole
    self terms do not depend on the positions."""
    pos, pp = _d(s.pos)
    n = pos.shape[0]
    _, ap = _d(s.alpha)
    _, tp = _d(s.thole)
    _, qp = _d(s.q)
    _, dp = _d(s.dip)
    _, Qp = _d(s.quad)
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1, 3))
    mp = mu.ctypes.data_as(_dp)
    _, sp = _i(s.sc_ptr)
    _, sjp = _i(s.sc_j if len(s.sc_j) else np.zeros(1, np.int32))
    _, ssp = _d(s.sc_s if len(s.sc_s) else np.zeros(1))
    if recip is None:
        bp, beta, rc = None, 0.0, math.inf
        cl = (None,) * 4
    else:
        _box, bp = _d(s.box)
        beta, rc = s.ewald_alpha, s.cutoff
        _cl, cl = _search_args(s, rc, search)
    n_out, _keep, ip = _outsel(n, idx)
    g = np.zeros((n_out, 3))
    lib().orc_polar_grad_real(n, pp, bp, beta, rc, ap, tp, qp, dp, Qp, mp, sp, sjp, ssp, n_out, ip,
                              g.ctypes.data_as(_dp), *cl)
    out = -COULOMB * g
    if recip == 'spme':
        psi_mu = spme_potential(s, spme_spread(s, dip=mu))
        psi_p = spme_potential(s, spme_spread(s, s.q, s.dip, s.quad))
        grid = tuple(s.grid)
        _g, gp = _i(np.asarray(grid, np.int32))
        _box, bp = _d(s.box)
        psa, psap = _d(psi_mu + psi_p)
        psb, psbp = _d(psi_mu)
        r = np.zeros((n_out, 3))
        lib().orc_spme_grad(n, pp, bp, gp, int(s.order), psap, psbp, mp, qp, dp, Qp, n_out, ip,
                            r.ctypes.data_as(_dp))
        out += COULOMB * r
    elif recip is not None:
        raise ValueError(recip)
    return out


def polar_energy(s, recip='spme', tol_debye=1e-12, dense=False):
    """E_pol (kcal/mol) at the exact dipoles of configuration s, and those dipoles."""
    e = perm_field(s, recip)
    if dense:
        mu = np.linalg.solve(dense_operator(s, recip), e.ravel()).reshape(-1, 3)
    else:
        mu, _, _ = pcg(s, e, recip, tol_debye=tol_debye, max_iter=5000)
    return e_pol(mu, e), mu
