"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
quadrature of the Thole smeared charge, explicit point-charge realisations of
multipoles, brute-force lattice sums, closed forms of small problems, Ewald
splitting invariance, symmetry, a dense textbook solve and the variational
identity of the polarization energy.  CPU only."""
import math

import numpy as np
import pytest
from scipy.integrate import quad as _quad
from scipy.linalg import cho_factor, cho_solve

import oracle as O
from paper_2011_01207_amd import synth


# ------------------------------------------------------------------------------------------
# helpers (independent of the oracle's closed forms)
# ------------------------------------------------------------------------------------------

def lam3_quadrature(r, ai, aj, a):
    """Charge fraction of the Thole density rho(u) ~ exp(-a u^3) enclosed within r
    (u = r / (ai aj)^(1/6)), by numerical quadrature of the normalised density."""
    u = r / (ai * aj) ** (1.0 / 6.0)
    val, _ = _quad(lambda x: 3.0 * a * x * x * np.exp(-a * x ** 3), 0.0, u, epsabs=1e-15, epsrel=1e-13,
                   limit=200)
    return val


def deriv4(f, r, h=1e-3):
    return (-f(r + 2 * h) + 8 * f(r + h) - 8 * f(r - h) + f(r - 2 * h)) / (12 * h)


def lam5_from_lam3(r, ai, aj, a):
    # The rank-2 tensor of the smeared-charge potential: its r r^T coefficient is
    # (3 l3 - r l3') / r^5 =: 3 l5 / r^5.
    f = lambda x: lam3_quadrature(x, ai, aj, a)
    return f(r) - r * deriv4(f, r) / 3.0


def lam7_from_lam5(r, ai, aj, a):
    g = lambda x: lam5_from_lam3(x, ai, aj, a)
    return g(r) - r * deriv4(g, r) / 5.0


def two_atom_system(r, alpha, a=0.39, q=(0.0, 0.0)):
    s = synth.tiny_cell(2, 100.0, 7, with_multipoles=False)
    s.pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    s.alpha = np.array([alpha, alpha])
    s.thole = np.array([a, a])
    s.q = np.array(q, dtype=float)
    return s


def small_water_box(seed=11):
    """27 waters on a 3^3 lattice (C1's spacing), rc = L/2, beta with a 1e-5 real-space tail."""
    s = synth.water_box(27, 9.315, 16, seed, "water_81")
    s.cutoff = 4.65
    s.ewald_alpha = 0.7
    return s


# ------------------------------------------------------------------------------------------
# P1: Thole damping
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0.6, 0.95, 1.5, 2.4, 3.5])
@pytest.mark.parametrize("ai,aj,a", [(0.837, 0.496, 0.39), (1.33, 0.84, 0.39), (0.5, 0.5, 0.2)])
def test_thole_lambdas_match_smeared_charge(r, ai, aj, a):
    l3, l5, l7 = O.thole_lambdas(r, ai, aj, a, a + 0.1)   # pair rule takes the smaller a
    assert abs(l3 - lam3_quadrature(r, ai, aj, a)) < 1e-12
    assert abs(l5 - lam5_from_lam3(r, ai, aj, a)) < 1e-9
    assert abs(l7 - lam7_from_lam5(r, ai, aj, a)) < 2e-7


def test_thole_limits():
    # far apart: no damping; at contact: finite (l3 ~ r^3, so l3/r^3 stays bounded)
    l3, l5, l7 = O.thole_lambdas(30.0, 0.8, 0.8, 0.39, 0.39)
    assert l3 == pytest.approx(1.0, abs=1e-15) and l5 == pytest.approx(1.0, abs=1e-15)
    ratios = [O.thole_lambdas(r, 0.8, 0.8, 0.39, 0.39)[0] / r ** 3 for r in (2e-2, 1e-2)]
    assert ratios[0] == pytest.approx(ratios[1], rel=1e-5)
    assert ratios[1] == pytest.approx(0.39 / 0.8, rel=1e-5)  # a / (alpha_i alpha_j)^(1/2)


@pytest.mark.parametrize("r", [1.2, 2.0, 3.0])
def test_two_atom_closed_form(r):
    """Two identical polarizable atoms in a uniform field (free space): along the axis
    mu = alpha E0 / (1 - alpha t_par), t_par = (3 l5 - l3)/r^3; across it
    mu = alpha E0 / (1 + alpha l3 / r^3).  l3, l5 by quadrature of the Thole density."""
    alpha, a = 0.837, 0.39
    s = two_atom_system(r, alpha, a)
    l3 = lam3_quadrature(r, alpha, alpha, a)
    l5 = lam5_from_lam3(r, alpha, alpha, a)
    op = lambda v: O.matvec(s, v, recip=None)
    for axis, expect in ((0, alpha / (1 - alpha * (3 * l5 - l3) / r ** 3)), (1, alpha / (1 + alpha * l3 / r ** 3))):
        e0 = np.zeros((2, 3))
        e0[:, axis] = 0.1
        mu, it, _ = O.pcg(s, e0, tol_debye=1e-14, op=op)
        assert mu[0, axis] == pytest.approx(0.1 * expect, rel=1e-8)
        assert mu[1, axis] == pytest.approx(0.1 * expect, rel=1e-8)
        assert it <= 3


# ------------------------------------------------------------------------------------------
# permanent-field kernels in free space
# ------------------------------------------------------------------------------------------

def _charges_field(point, charges):
    e = np.zeros(3)
    for qk, sk in charges:
        d = point - sk
        e += qk * d / np.linalg.norm(d) ** 3
    return e


def test_free_space_dipole_and_quadrupole_match_point_charges():
    """Field of a point dipole and a traceless quadrupole (potential Theta:rr/r^5) equals the
    field of explicit point charges with those moments (dipole: +-q at +-h/2; quadrupole:
    three linear quadrupoles along the eigenvectors of Theta), to O(h^2)."""
    rng = np.random.default_rng(3)
    s = two_atom_system(2.7, 0.8, a=1e9)   # Thole a huge: no damping at this distance
    s.pos[1] = np.array([1.9, -1.1, 1.4])
    dip, quad6 = synth.random_multipoles(rng, 2)
    s.q = np.zeros(2)
    h = 1e-3
    # dipole
    s.dip = np.zeros((2, 3)); s.dip[0] = dip[0]; s.quad = np.zeros((2, 6))
    e_or = O.real_perm(s, idx=[1], free_space=True)[0]
    u = dip[0] / np.linalg.norm(dip[0])
    qd = np.linalg.norm(dip[0]) / h
    ch = [(qd, s.pos[0] + 0.5 * h * u), (-qd, s.pos[0] - 0.5 * h * u)]
    e_ch = _charges_field(s.pos[1], ch)
    assert np.allclose(e_or, e_ch, rtol=1e-6, atol=1e-9)
    # quadrupole
    t = quad6[0]
    th = np.array([[t[0], t[1], t[2]], [t[1], t[3], t[4]], [t[2], t[4], t[5]]])
    s.dip = np.zeros((2, 3)); s.quad = np.zeros((2, 6)); s.quad[0] = t
    e_or = O.real_perm(s, idx=[1], free_space=True)[0]
    w, v = np.linalg.eigh(th)
    ch = []
    for k in range(3):
        c = w[k] / (3 * h * h)
        e = v[:, k]
        ch += [(c, s.pos[0] + h * e), (c, s.pos[0] - h * e), (-2 * c, s.pos[0])]
    e_ch = _charges_field(s.pos[1], ch)
    assert np.allclose(e_or, e_ch, rtol=1e-5, atol=1e-9)


def test_free_space_charge_field_thole_damped_and_scaled():
    r, alpha, a = 1.3, 0.9, 0.39
    s = two_atom_system(r, alpha, a, q=(0.0, 0.7))
    s.dip = np.zeros((2, 3)); s.quad = np.zeros((2, 6))
    e = O.real_perm(s, idx=[0], free_space=True, scaled=False)[0]
    l3 = lam3_quadrature(r, alpha, alpha, a)
    assert e[0] == pytest.approx(-0.7 * l3 / r ** 2, rel=1e-10)
    # scale 0 removes the pair completely in free space; scale 0.5 halves it
    for sc in (0.0, 0.5):
        s.sc_ptr = np.array([0, 1, 2], np.int32)
        s.sc_j = np.array([1, 0], np.int32)
        s.sc_s = np.array([sc, sc])
        e2 = O.real_perm(s, idx=[0], free_space=True)[0]
        assert e2[0] == pytest.approx(sc * e[0], abs=1e-15)


# ------------------------------------------------------------------------------------------
# P2-P4: Ewald sum
# ------------------------------------------------------------------------------------------

def _beta_system():
    s = synth.tiny_cell(16, 24.0, 21, min_dist=1.3)
    s.cutoff = 12.0
    # a few scaled pairs so that the correction's reciprocal share is exercised
    pairs = [(0, 1, 0.0), (2, 3, 0.5), (4, 5, 0.0)]
    ptr, sj, ss = synth.build_csr(16, [(i, j) for i, j, _ in pairs], [x for _, _, x in pairs])
    s.sc_ptr, s.sc_j, s.sc_s = ptr, sj, ss
    return s


def test_ewald_beta_invariance_mutual_and_permanent():
    s = _beta_system()
    mu = np.random.default_rng(9).standard_normal((16, 3)) * 0.1
    fm, fp = [], []
    for beta in (0.5, 0.6, 0.75, 0.9):
        fm.append(O.mutual_field(s, mu, 'ksum', beta=beta))
        fp.append(O.perm_field(s, 'ksum', beta=beta))
    for f in (fm, fp):
        scale = np.abs(f[0]).max()
        for g in f[1:]:
            assert np.abs(g - f[0]).max() < 1e-11 * scale


@pytest.mark.parametrize("sep", [2.2, 4.5])
def test_exclusion_removes_exactly_the_pair(sep):
    """Excluding a pair (scale 0) must change the periodic field at its atoms by exactly the
    pair's direct damped interaction (minimum image), whether the pair lies inside the
    real-space cutoff (3 A) or beyond it; a half scale removes half of it."""
    s = synth.tiny_cell(8, 12.0, 33, min_dist=1.5)
    s.pos[1] = (s.pos[0] + np.array([sep, 0.0, 0.0])) % 12.0
    s.cutoff, s.ewald_alpha = 3.0, 2.0
    full = O.perm_field(s, 'ksum')
    two = synth.tiny_cell(2, 100.0, 1)
    two.pos = np.array([[0.0, 0.0, 0.0], [sep, 0.0, 0.0]])
    for f in ("alpha", "thole", "q", "dip", "quad"):
        setattr(two, f, getattr(s, f)[:2].copy())
    direct = O.real_perm(two, idx=[0, 1], free_space=True, scaled=False)
    for sc in (0.0, 0.5):
        ptr, sj, ss = synth.build_csr(8, [(0, 1)], [sc])
        s.sc_ptr, s.sc_j, s.sc_s = ptr, sj, ss
        ex = O.perm_field(s, 'ksum')
        assert np.allclose(full[:2] - ex[:2], (1 - sc) * direct, rtol=1e-9, atol=1e-12)
        assert np.allclose(full[2:], ex[2:], rtol=1e-12, atol=1e-14)
        s.sc_ptr, s.sc_j, s.sc_s = np.zeros(9, np.int32), np.zeros(0, np.int32), np.zeros(0)


def _brute_dipole_lattice(s, mu, radius):
    L = s.box[0]
    m = int(np.ceil(radius))
    g = np.arange(-m, m + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)
    n = n[np.linalg.norm(n, axis=1) <= radius]
    out = np.zeros_like(mu)
    for i in range(len(mu)):
        for j in range(len(mu)):
            r = s.pos[i] - s.pos[j] - n * L
            if i == j:
                r = r[np.any(n != 0, axis=1)]
            rr = np.linalg.norm(r, axis=1)
            mr = r @ mu[j]
            out[i] += (3 * mr[:, None] * r / rr[:, None] ** 5 - mu[j] / rr[:, None] ** 3).sum(0)
    return out


@pytest.mark.parametrize("net", [False, True])
def test_ewald_matches_spherical_lattice_sum(net):
    """Direct sum over periodic images in growing spheres (vacuum outside) equals the tin-foil
    Ewald field minus the Lorentz term 4 pi M / (3 V) of the net cell dipole M."""
    s = synth.tiny_cell(4, 10.0, 101, min_dist=3.5)
    s.thole[:] = 1e9
    s.cutoff, s.ewald_alpha = 5.0, 1.2
    mu = np.random.default_rng(5).standard_normal((4, 3)) * 0.1
    if not net:
        mu -= mu.mean(0)
    ew = O.mutual_field(s, mu, 'ksum')
    ref = ew - (4 * np.pi / (3 * 1000.0)) * mu.sum(0)
    brute = _brute_dipole_lattice(s, mu, 40)
    assert np.abs(brute - ref).max() < 2e-7 * np.abs(ref).max()


def test_single_atom_in_cubic_box():
    """One polarizable atom: its periodic images give (tin-foil) exactly 4 pi mu / (3 L^3),
    so mu = alpha E0 / (1 - 4 pi alpha / (3 L^3)).  The k-sum reproduces it to rounding;
    smooth PME approaches it as the grid is refined."""
    L, alpha = 10.0, 1.0
    s = synth.tiny_cell(1, L, 3, with_multipoles=False)
    s.pos = np.array([[1.3, 4.1, 7.7]])
    s.alpha = np.array([alpha])
    s.cutoff, s.ewald_alpha = 5.0, 0.8
    e0 = np.array([[0.1, -0.05, 0.02]])
    expect = alpha * e0 / (1 - 4 * np.pi * alpha / (3 * L ** 3))
    mu, _, _ = O.pcg(s, e0, 'ksum', tol_debye=1e-14)
    assert np.allclose(mu, expect, rtol=1e-12, atol=0)
    errs = []
    for K in (16, 32, 64):
        s.grid = (K, K, K)
        mu, _, _ = O.pcg(s, e0, 'spme', tol_debye=1e-14)
        errs.append(np.abs(mu - expect).max())
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4 and errs[2] < 1e-6


# ------------------------------------------------------------------------------------------
# P5-P7: operator symmetry, dense solve, variational identity
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("recip", ["ksum", "spme"])
def test_operator_symmetric(recip):
    s = synth.water648()
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, s.n, 3)) * 0.1
    a = np.sum(u * O.mutual_field(s, v, recip))
    b = np.sum(v * O.mutual_field(s, u, recip))
    assert abs(a - b) < 1e-12 * max(abs(a), abs(b))


def test_dense_operator_spd_and_cholesky_equals_pcg():
    s = small_water_box()
    a = O.dense_operator(s, 'spme')
    assert np.abs(a - a.T).max() < 1e-12 * np.abs(a).max()
    assert np.linalg.eigvalsh(0.5 * (a + a.T)).min() > 0
    e = O.perm_field(s, 'spme')
    mu_chol = cho_solve(cho_factor(a), e.ravel()).reshape(-1, 3)
    mu_pcg, it, _ = O.pcg(s, e, 'spme', tol_debye=1e-12)
    assert O.rms_debye(mu_pcg - mu_chol) < 1e-10


def test_variational_identity_and_energy():
    s = small_water_box()
    e = O.perm_field(s, 'spme')
    mu, _, _ = O.pcg(s, e, 'spme', tol_debye=1e-12)
    U = lambda m: 0.5 * np.sum(m * O.matvec(s, m, 'spme')) - np.sum(m * e)
    # U at the solution equals -1/2 mu.E, i.e. E_pol / C
    assert O.e_pol(mu, e) == pytest.approx(O.COULOMB * U(mu), rel=1e-10)
    rng = np.random.default_rng(2)
    for _ in range(3):
        d = rng.standard_normal(mu.shape) * 1e-2
        du = U(mu + d) - U(mu)
        assert du > 0
        assert du == pytest.approx(0.5 * np.sum(d * O.matvec(s, d, 'spme')), rel=1e-7)
    # the energy functional decreases monotonically along CG iterates
    us = []
    for k in range(1, 8):
        m, _, _ = O.pcg(s, e, 'spme', tol_debye=0.0, max_iter=k)
        us.append(U(m))
    assert all(b < a + 1e-15 for a, b in zip(us, us[1:]))


# ------------------------------------------------------------------------------------------
# P8: smooth PME converges to the exact Ewald sum
# ------------------------------------------------------------------------------------------

def test_spme_converges_to_ksum():
    s = synth.water648()
    mu = np.random.default_rng(0).standard_normal((s.n, 3)) * 0.05
    ek_mu = O.ksum_field(s, dip=mu)
    ek_pm = O.ksum_field(s, q=s.q, dip=s.dip, quad=s.quad)
    errs_mu, errs_pm = [], []
    for K in (16, 24, 32, 48, 64, 96):
        errs_mu.append(np.sqrt(np.mean((O.spme_field(s, dip=mu, grid=(K,) * 3) - ek_mu) ** 2)))
        errs_pm.append(np.sqrt(np.mean((O.spme_field(s, s.q, s.dip, s.quad, grid=(K,) * 3) - ek_pm) ** 2)))
    for errs, ref, bar in ((errs_mu, ek_mu, 1e-5), (errs_pm, ek_pm, 5e-5)):
        assert all(b < a for a, b in zip(errs, errs[1:]))
        assert errs[-1] < bar * np.sqrt(np.mean(ref ** 2))
        assert errs[-1] < 2e-3 * errs[0]


def test_bspline_partition_of_unity_and_moduli():
    # sum_k M_n(x + k) = 1 and sum_k M_n'(x + k) = 0 for any x (cardinal B-spline facts)
    for x in (0.0, 0.137, 0.5, 0.93):
        assert sum(O.bspline(5, x + k) for k in range(5)) == pytest.approx(1.0, abs=1e-15)
        assert sum(O.bspline(5, x + k, 1) for k in range(5)) == pytest.approx(0.0, abs=1e-14)
        assert sum(O.bspline(5, x + k, 2) for k in range(5)) == pytest.approx(0.0, abs=1e-13)
    # order-5 knot values 1/24, 11/24, 11/24, 1/24
    assert [O.bspline(5, k) for k in (1, 2, 3, 4)] == pytest.approx([1 / 24, 11 / 24, 11 / 24, 1 / 24], abs=1e-15)


# ------------------------------------------------------------------------------------------
# P12: generators
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [synth.water648, synth.solvated_chain])
def test_generator_invariants(maker):
    s = maker()
    assert abs(s.q.sum()) < 1e-10
    assert np.all(s.pos >= 0) and np.all(s.pos < s.box)
    assert np.allclose(s.quad[:, 0] + s.quad[:, 3] + s.quad[:, 5], 0.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(s.dip, axis=1), 0.1)
    nw = s.meta["n_waters"]
    first = s.n - 3 * nw
    o = s.pos[first::3]
    for k in (1, 2):
        d = s.pos[first + k::3] - o
        d -= s.box * np.round(d / s.box)
        assert np.allclose(np.linalg.norm(d, axis=1), 0.9572, atol=1e-12)
    d1 = s.pos[first + 1::3] - o
    d2 = s.pos[first + 2::3] - o
    d1 -= s.box * np.round(d1 / s.box)
    d2 -= s.box * np.round(d2 / s.box)
    ang = np.degrees(np.arccos(np.sum(d1 * d2, 1) / (0.9572 ** 2)))
    assert np.allclose(ang, 104.52, atol=1e-9)
    # CSR symmetric, no self pairs
    for i in range(0, s.n, max(1, s.n // 500)):
        for k in range(s.sc_ptr[i], s.sc_ptr[i + 1]):
            j = s.sc_j[k]
            assert j != i
            row = s.sc_j[s.sc_ptr[j]:s.sc_ptr[j + 1]]
            assert i in row
    # seed reproducibility
    t = maker()
    assert np.array_equal(s.pos, t.pos) and np.array_equal(s.dip, t.dip)


def test_generator_counts():
    s = synth.water648()
    assert s.n == 648 and s.sc_ptr[-1] == 2 * 648
    c = synth.solvated_chain()
    assert c.n == 23558 == 2489 + 3 * 7023
    assert c.sc_ptr[-1] == 2 * 28530
    assert np.count_nonzero(c.sc_s == 0.5) == 2 * 2486


# ------------------------------------------------------------------------------------------
# pair counting and partner search
# ------------------------------------------------------------------------------------------

# Number of integer vectors (i, j, k) with i^2 + j^2 + k^2 = m (sums of three squares): the
# coordination shells of the simple cubic lattice.  m = 7 has no representation.
R3 = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24, 7: 0, 8: 12, 9: 30, 10: 24}


def cubic_lattice(n_edge, spacing, seed=0, shift=0.0):
    s = synth.tiny_cell(2, n_edge * spacing, seed, with_multipoles=False)
    g = np.arange(n_edge) * spacing + shift
    s.pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    s.box = np.full(3, n_edge * spacing)
    return s


@pytest.mark.parametrize("search", ["all", "cells"])
@pytest.mark.parametrize("rc2, shells", [(6.5, 6), (5.0, 4), (9.5, 9), (2.0, 1)])
def test_pair_count_on_cubic_lattice(search, rc2, shells):
    """Unordered pairs within rc of a periodic simple cubic lattice: N/2 times the lattice
    vectors with |v| < rc.  rc^2 = 5 a^2 puts rc exactly on the fifth shell (sqrt(20) and
    2 sqrt(5) are the same double), which the strict r < rc must leave out; shells wrapping
    through the faces are counted only with the minimum image."""
    a, n_edge = 2.0, 8
    s = cubic_lattice(n_edge, a, shift=0.375)   # exact in binary: lattice differences stay exact
    rc = a * math.sqrt(rc2)
    per_atom = sum(R3[m] for m in R3 if m <= shells and m < rc2)
    assert O.count_pairs(s, rc=rc, search=search) == n_edge ** 3 * per_atom // 2


def test_cell_search_finds_the_same_pairs_as_all_pairs():
    """The periodic cell grid (at least three cells of width >= rc per axis) finds every pair
    within rc: same counts, and the same fields up to the order of the sums, on a box with atoms
    placed on the cell faces and in the solvated chain with its scaled pairs."""
    s = synth.tiny_cell(300, 22.0, 5, min_dist=0.8)
    # atoms exactly on the cell boundaries (multiples of L/3) and at the box edge
    s.pos[:6] = [[0.0, 0.0, 0.0], [22.0 / 3, 5.0, 5.0], [44.0 / 3, 44.0 / 3, 1.0], [21.999999, 3.0, 7.0],
                 [7.0, 22.0 / 3 + 7.0, 3.0], [11.0, 11.0, 22.0 / 3]]
    assert O.cell_bins(s.pos, s.box, s.cutoff) is not None
    assert O.count_pairs(s, search="cells") == O.count_pairs(s, search="all")
    rng = np.random.default_rng(3)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    a = O.real_mutual(s, mu, search="cells")
    b = O.real_mutual(s, mu, search="all")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    c = synth.solvated_chain()
    idx = np.sort(rng.choice(c.n, 1500, replace=False))
    assert O.count_pairs(c, search="cells") == O.count_pairs(c, search="all")
    a = O.real_perm(c, idx=idx, search="cells")
    b = O.real_perm(c, idx=idx, search="all")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    mu = rng.standard_normal((c.n, 3)) * 0.05
    a = O.real_mutual(c, mu, idx=idx, search="cells")
    b = O.real_mutual(c, mu, idx=idx, search="all")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_unit_constants_from_si():
    """Debye per e*A and the Coulomb constant in kcal*A/(mol e^2), from the exact SI values of
    e, c, N_A and the thermochemical calorie, and CODATA 2018 epsilon_0."""
    e, c, na, eps0 = 1.602176634e-19, 299792458.0, 6.02214076e23, 8.8541878128e-12
    debye = e * 1e-10 / (1e-21 / c)          # e*A in C*m over 1 D = 1e-21/c C*m
    assert O.DEBYE == pytest.approx(debye, rel=2e-6)
    coulomb = e * e / (4 * math.pi * eps0) * 1e10 * na / 4184.0
    assert O.COULOMB == pytest.approx(coulomb, rel=2e-7)
