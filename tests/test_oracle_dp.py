"""Pins of the oracle's two-set (d/p) model, CPU only.

* The two permanent fields differ only through the listed pairs whose direct and polarization
  scales differ, each by (s_d - s_p) times the pair's bare Thole-damped field, which is evaluated
  here pair by pair as the free-space field of a two-atom system (no Ewald split, no cutoff).
* With the direct scales equal to the p-scales both fields are the same array.
* The operator is symmetric, so mu_d . E_p = mu_p . E_d for the exact solutions (dense solve of a
  small system), which is the two-set energy's consistency; PCG reaches the same solutions."""
import types

import numpy as np

import oracle as O
from paper_2011_01207_amd import synth


def tiny_chain():
    # 30 chain atoms + 60 waters in a 16 A box (cutoff 7 A < L/2), grid 16^3
    return synth.solvated_chain(seed=21, box_len=16.0, n_chain=30, n_w=60, lattice=5, grid=16,
                                name="solvated_chain_210")


def pair_field(s, i, j):
    """Bare field at atom i of atom j's multipoles (minimum image), as the free-space field of
    the two-atom system {i, j} with no scaled pairs."""
    L = np.asarray(s.box, dtype=np.float64)
    d = s.pos[j] - s.pos[i]
    d -= L * np.round(d / L)
    two = types.SimpleNamespace(
        pos=np.stack([s.pos[i], s.pos[i] + d]), box=L, alpha=s.alpha[[i, j]], thole=s.thole[[i, j]],
        q=s.q[[i, j]], dip=s.dip[[i, j]], quad=s.quad[[i, j]], sc_ptr=np.zeros(3, np.int32),
        sc_j=np.zeros(0, np.int32), sc_s=np.zeros(0), cutoff=s.cutoff, ewald_alpha=s.ewald_alpha,
        grid=s.grid, order=s.order)
    return O.real_perm(two, free_space=True, scaled=False)[0]


def test_dp_fields_differ_by_the_pairs_whose_scales_differ():
    s = synth.solvated_chain_small()
    e_d, e_p = O.perm_field_dp(s, "spme")
    expect = np.zeros_like(e_p)
    rows = np.repeat(np.arange(s.n), np.diff(s.sc_ptr))
    diff = s.sc_s_d - s.sc_s
    assert np.count_nonzero(diff) > 100
    for k in np.nonzero(diff)[0]:
        expect[rows[k]] += diff[k] * pair_field(s, rows[k], s.sc_j[k])
    got = e_d - e_p
    scale = np.max(np.abs(e_p))
    assert np.max(np.abs(got - expect)) < 1e-11 * scale, np.max(np.abs(got - expect))
    # atoms with no differing pair: identical fields
    touched = np.zeros(s.n, bool)
    touched[rows[diff != 0]] = True
    assert np.array_equal(e_d[~touched], e_p[~touched])


def test_dp_reduces_to_one_set_when_the_scales_agree():
    s = tiny_chain()
    s.sc_s_d = s.sc_s.copy()
    e_d, e_p = O.perm_field_dp(s, "spme")
    assert np.array_equal(e_d, e_p)
    w = synth.water648()
    e_d, e_p = O.perm_field_dp(w, "spme")
    assert np.array_equal(e_d, e_p)
    assert np.array_equal(e_p, O.perm_field(w, "spme"))


def test_two_set_energy_is_symmetric():
    s = tiny_chain()
    e_d, e_p = O.perm_field_dp(s, "spme")
    a = O.dense_operator(s, "spme")
    mu_d = np.linalg.solve(a, e_d.reshape(-1)).reshape(-1, 3)
    mu_p = np.linalg.solve(a, e_p.reshape(-1)).reshape(-1, 3)
    u_dp, u_pd = O.e_pol_dp(mu_d, e_p), O.e_pol_dp(mu_p, e_d)
    assert abs(u_dp - u_pd) < 1e-10 * abs(u_dp)
    assert abs(u_dp - O.e_pol(mu_p, e_p)) > 1e-6 * abs(u_dp)  # the two sets really differ
    # PCG of either set reaches the dense solution
    for rhs, ref in ((e_d, mu_d), (e_p, mu_p)):
        mu, it, _ = O.pcg(s, rhs, "spme", tol_debye=1e-10)
        assert O.rms_debye(mu - ref) < 1e-8
