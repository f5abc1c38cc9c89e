"""Pins of the oracle's polarization energy gradient (CPU).

At the converged dipoles the polarization energy is stationary in mu, so its gradient with
respect to the positions follows from the pair tensors and the spline derivatives alone.  Each
pin compares that analytic gradient with central differences of the oracle's own E_pol, solved
exactly (dense linear solve) at the displaced positions: nothing else from the oracle enters
the comparison, and a wrong sign, factor, damping function (lambda9 included) or spline
derivative shows as a difference far above the O(h^2) of the differences."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2011_01207_amd import synth


def cluster(n_w=4, s13=0.0):
    """The first n_w waters of the 648-atom box as a free-space cluster (neutral, with the
    intramolecular pairs: O-H excluded, H-H scaled by s13)."""
    base = synth.water648()
    n = 3 * n_w
    s = copy.deepcopy(base)
    s.pos = base.pos[:n].copy()
    s.q = base.q[:n] - base.q[:n].mean()
    s.dip, s.quad = base.dip[:n].copy(), base.quad[:n].copy()
    s.alpha, s.thole = base.alpha[:n].copy(), base.thole[:n].copy()
    pairs, scales = [], []
    for i in range(n):
        for k in range(base.sc_ptr[i], base.sc_ptr[i + 1]):
            j = int(base.sc_j[k])
            if j < n and i < j:
                pairs.append((i, j))
                scales.append(s13 if (i % 3 and j % 3) else float(base.sc_s[k]))
    s.sc_ptr, s.sc_j, s.sc_s = synth.build_csr(n, pairs, scales)
    return s


def central_difference(s, recip, coords, h=1e-5):
    out = []
    for a, c in coords:
        e = []
        for sign in (1.0, -1.0):
            d = copy.deepcopy(s)
            d.pos = s.pos.copy()
            d.pos[a, c] += sign * h
            e.append(O.polar_energy(d, recip, dense=True)[0])
        out.append((e[0] - e[1]) / (2 * h))
    return np.array(out)


def test_free_space_gradient_matches_central_differences():
    """Four waters in free space: every coordinate of every atom."""
    s = cluster()
    _, mu = O.polar_energy(s, None, dense=True)
    g = O.polar_gradient(s, mu, None)
    coords = [(a, c) for a in range(s.n) for c in range(3)]
    num = central_difference(s, None, coords)
    ana = np.array([g[a, c] for a, c in coords])
    assert np.max(np.abs(ana - num)) < 1e-7 * np.max(np.abs(num))


def test_free_space_gradient_with_partial_scaling():
    """O-H pairs excluded, H-H pairs scaled by 0.5 (both terms of the scale enter)."""
    s = cluster(3, s13=0.5)
    assert sorted(set(np.round(s.sc_s, 6))) == [0.0, 0.5]
    _, mu = O.polar_energy(s, None, dense=True)
    g = O.polar_gradient(s, mu, None)
    coords = [(a, c) for a in range(s.n) for c in range(3)]
    num = central_difference(s, None, coords)
    ana = np.array([g[a, c] for a, c in coords])
    assert np.max(np.abs(ana - num)) < 1e-7 * np.max(np.abs(num))


@pytest.mark.parametrize("rc", [4.65, 1.45])
def test_periodic_spme_gradient_matches_central_differences(rc):
    """27 waters in a periodic box, smooth PME on a 16^3 grid, random coordinates.  With
    rc = 1.45 A the excluded H-H pairs (1.51 A) lie beyond the cutoff, so the correction of
    listed pairs outside rc is exercised as well."""
    s = synth.water_box(27, 9.315, 16, 11, "water_81")
    s.cutoff = rc
    s.ewald_alpha = 0.7
    _, mu = O.polar_energy(s, "spme", dense=True)
    g = O.polar_gradient(s, mu, "spme")
    rng = np.random.default_rng(int(rc * 100))
    coords = [(int(rng.integers(s.n)), int(rng.integers(3))) for _ in range(8)]
    num = central_difference(s, "spme", coords)
    ana = np.array([g[a, c] for a, c in coords])
    assert np.max(np.abs(ana - num)) < 1e-7 * np.max(np.abs(g))


def test_gradient_partner_search_and_sampling_agree():
    """Cell search equals all pairs; a sample of atoms equals the full evaluation at the sample."""
    s = synth.solvated_chain()
    rng = np.random.default_rng(9)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    idx = np.sort(rng.choice(s.n, 800, replace=False))
    a = O.polar_gradient(s, mu, "spme", idx=idx)
    b = O.polar_gradient(s, mu, "spme", idx=idx, search="all")
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    small = synth.water648()
    mu = rng.standard_normal((small.n, 3)) * 0.05
    full = O.polar_gradient(small, mu, "spme")
    idx = np.array([0, 5, 17, 300, 647])
    assert np.max(np.abs(O.polar_gradient(small, mu, "spme", idx=idx) - full[idx])) <= 1e-13 * np.max(np.abs(full))
