"""GPU parity of every kernel stage against the FP64 oracle, through the C ABI.

FP64 mode must agree with the oracle's smooth-PME evaluation (same grid, order, beta, cutoff)
to rounding; mixed precision (FP32 pair/PME math, fixed-point accumulation, FP64 PCG) to the
stated bounds.  Discretization error of PME against the exact Ewald k-sum is measured by the
oracle tests, not here."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2011_01207_amd import amoeba, synth
from parity_util import assert_fields  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"




def tiny_water(n_w, L, K, seed, rc=None):
    s = synth.water_box(n_w, L, K, seed, f"water_{3 * n_w}")
    if rc is not None:
        s.cutoff = rc
    return s


@pytest.fixture(scope="module")
def c1():
    return synth.water648()


@pytest.fixture(scope="module")
def c1_ref(c1):
    rng = np.random.default_rng(42)
    mu = rng.standard_normal((c1.n, 3)) * 0.05
    return {
        "mu": mu,
        "real": O.real_mutual(c1, mu),
        "recip": O.spme_field(c1, dip=mu),
        "matvec": O.matvec(c1, mu, "spme"),
        "perm": O.perm_field(c1, "spme"),
    }


@pytest.fixture(scope="module", params=["fp64", "mixed"])
def c1_ctx(request, c1):
    print(f"[gpu] c1 context {request.param}", flush=True)
    ctx, t = amoeba.context_for(c1, precision=request.param, device=DEV)
    yield request.param, ctx, t
    ctx.close()


TOL = {"fp64": {"real": 1e-12, "recip": 1e-11, "matvec": 1e-12, "perm": 1e-11},
       "mixed": {"real": 2e-6, "recip": 2e-5, "matvec": 2e-6, "perm": 2e-5}}


def test_pair_count_equals_oracle(c1, c1_ctx):
    prec, ctx, t = c1_ctx
    assert ctx.info()["n_pairs"] == O.count_pairs(c1)


def test_real_and_recip_fields(c1, c1_ref, c1_ctx):
    prec, ctx, t = c1_ctx
    mu = torch.tensor(c1_ref["mu"], device=DEV)
    er, ek = ctx.dipole_field_parts(t["pos"], mu)
    assert_fields(er.cpu().numpy(), c1_ref["real"], TOL[prec]["real"])
    assert_fields(ek.cpu().numpy(), c1_ref["recip"], TOL[prec]["recip"])


def test_matvec(c1, c1_ref, c1_ctx):
    prec, ctx, t = c1_ctx
    mu = torch.tensor(c1_ref["mu"], device=DEV)
    out = ctx.dipole_matvec(t["pos"], mu).cpu().numpy()
    assert_fields(out, c1_ref["matvec"], TOL[prec]["matvec"])


def test_perm_field(c1, c1_ref, c1_ctx):
    prec, ctx, t = c1_ctx
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]).cpu().numpy()
    assert_fields(e, c1_ref["perm"], TOL[prec]["perm"])


def test_polarize_c1(c1, c1_ref, c1_ctx):
    prec, ctx, t = c1_ctx
    e_ref = c1_ref["perm"]
    mu_ref, it_ref, _ = O.pcg(c1, e_ref, "spme", tol_debye=1e-10)
    e_gpu = torch.tensor(e_ref, device=DEV)
    mu, ep, it, st = ctx.polarize(t["pos"], e_gpu, tol_debye=1e-7, max_iter=200)
    assert st == amoeba.AMOEBA_OK
    err = O.rms_debye(mu.cpu().numpy() - mu_ref)
    ep_ref = O.e_pol(mu_ref, e_ref)
    if prec == "fp64":
        assert err < 2e-7
        assert abs(ep - ep_ref) < 1e-8 * abs(ep_ref)
        # same iteration count as the oracle's PCG at the configuration's own tolerance
        _, it_o, _ = O.pcg(c1, e_ref, "spme", tol_debye=1e-6)
        _, _, it_g, _ = ctx.polarize(t["pos"], e_gpu, tol_debye=1e-6, max_iter=200)
        assert abs(it_g - it_o) <= 1
    else:
        assert err < 1e-5
        assert abs(ep - ep_ref) < 1e-5 * abs(ep_ref)


def test_mixed_solve_is_bitwise_deterministic(c1):
    ctx, t = amoeba.context_for(c1, precision="mixed", device=DEV)
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    a, ea, ia, _ = ctx.polarize(t["pos"], e, tol_debye=1e-6)
    b, eb, ib, _ = ctx.polarize(t["pos"], e, tol_debye=1e-6)
    assert torch.equal(a, b) and ea == eb and ia == ib
    # a fresh context (fresh list build) gives the same bits
    ctx2, t2 = amoeba.context_for(c1, precision="mixed", device=DEV)
    e2 = ctx2.perm_field(t2["pos"], t2["q"], t2["dip"], t2["quad"])
    assert torch.equal(e, e2)
    c, ec, ic, _ = ctx2.polarize(t2["pos"], e2, tol_debye=1e-6)
    assert torch.equal(a, c)
    ctx.close()
    ctx2.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solvated_chain_perm_and_matvec(prec):
    """23,558 atoms with 1-2/1-3 exclusions and 1-4 half scaling; compared at sampled atoms."""
    s = synth.solvated_chain()
    print(f"[gpu] solvated chain {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(s.n, 300, replace=False))
    idx = np.unique(np.concatenate([idx, np.arange(0, 40)]))   # include chain atoms with 1-4 pairs
    e_ref = O.perm_field(s, "spme", idx=idx)
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]).cpu().numpy()[idx]
    tol = 1e-11 if prec == "fp64" else 3e-5
    assert_fields(e, e_ref, tol)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    q_ref = O.matvec(s, mu, "spme", idx=idx)
    q = ctx.dipole_matvec(t["pos"], torch.tensor(mu, device=DEV)).cpu().numpy()[idx]
    assert_fields(q, q_ref, (1e-12 if prec == "fp64" else 3e-6))
    ctx.close()


def test_ragged_single_block_and_no_scaled_pairs():
    """Fewer atoms than one block (phantom padding), no scaled pairs, non-cubic box."""
    s = synth.tiny_cell(37, 16.0, 5, min_dist=1.2)
    s.box = np.array([16.0, 17.0, 18.5])
    s.pos = np.mod(s.pos, s.box)
    s.cutoff, s.ewald_alpha, s.grid = 6.0, 0.6, (20, 18, 25)
    ctx, t = amoeba.context_for(s, precision="fp64", device=DEV)
    assert ctx.info()["n_pairs"] == O.count_pairs(s)
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]).cpu().numpy()
    assert_fields(e, O.perm_field(s, "spme"), 1e-11)
    mu_ref, _, _ = O.pcg(s, O.perm_field(s, "spme"), "spme", tol_debye=1e-10)
    mu, _, _, st = ctx.polarize(t["pos"], torch.tensor(e, device=DEV), tol_debye=1e-9)
    assert st == amoeba.AMOEBA_OK and O.rms_debye(mu.cpu().numpy() - mu_ref) < 1e-8
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_near_coincident_atoms(prec):
    """Pairs at 0.02, 0.1, 0.3 and 0.45 A (the short-range series of the FP32 kernels) and
    their multipoles: real-space field, matvec, permanent field and a converged solve against
    the oracle."""
    import dataclasses
    s = synth.tiny_cell(40, 16.0, seed=140, min_dist=1.2)
    pos = s.pos.copy()
    for (i, j), d in zip(((0, 1), (2, 3), (4, 5), (6, 7)), (0.02, 0.1, 0.3, 0.45)):
        v = np.array([0.6, -0.48, 0.64])
        pos[j] = np.mod(pos[i] + d * v, 16.0)
    s = dataclasses.replace(s, pos=pos, grid=(20, 20, 20))
    rng = np.random.default_rng(141)
    mu = rng.standard_normal((s.n, 3)) * 0.05
    print(f"[gpu] near-coincident atoms {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    mt = torch.tensor(mu, device=DEV)
    # FP64: the direct formulas of both sides cancel at 0.02 A (B2 ~ 3/r^5 ~ 1e9), ~1e-10 relative
    tf = 1e-9 if prec == "fp64" else 2e-6
    er, _ = ctx.dipole_field_parts(t["pos"], mt)
    assert_fields(er.cpu().numpy(), O.real_mutual(s, mu), tf, what="real field")
    assert_fields(ctx.dipole_matvec(t["pos"], mt).cpu().numpy(), O.matvec(s, mu, "spme"), tf, what="matvec")
    e_ref = O.perm_field(s, "spme")
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    # FP64 permanent field: B3 ~ 15/r^7 ~ 1e13 at 0.02 A cancels in both direct formulas
    assert_fields(e.cpu().numpy(), e_ref, 1e-7 if prec == "fp64" else 2e-5, what="E_perm")
    mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-10)
    m, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-7 if prec == "fp64" else 1e-6)
    assert st == amoeba.AMOEBA_OK
    err = O.rms_debye(m.cpu().numpy() - mu_ref)
    assert err < (3e-7 if prec == "fp64" else 5e-6), err
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_atom(prec):
    """One atom in a 16 A box: no pairs, one block of 63 phantoms, only the reciprocal and self
    terms act on it (its periodic images)."""
    import dataclasses
    s = dataclasses.replace(synth.tiny_cell(1, 16.0, 7), grid=(16, 16, 16))
    print(f"[gpu] single atom {prec}", flush=True)
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        assert ctx.info()["n_pairs"] == 0
        e_ref = O.perm_field(s, "spme")
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        assert_fields(e.cpu().numpy(), e_ref, (1e-11 if prec == "fp64" else 3e-5))
        mu = np.full((1, 3), 0.1)
        q = ctx.dipole_matvec(t["pos"], torch.tensor(mu, device=DEV)).cpu().numpy()
        assert_fields(q, O.matvec(s, mu, "spme"), (1e-12 if prec == "fp64" else 3e-6))
        mu_ref, _, _ = O.pcg(s, e_ref, "spme", tol_debye=1e-10)
        m, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-9 if prec == "fp64" else 1e-7)
        assert st == amoeba.AMOEBA_OK
        assert O.rms_debye(m.cpu().numpy() - mu_ref) < (1e-8 if prec == "fp64" else 1e-6)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_permanent_field_converges_at_the_start(prec):
    """E_perm = 0: the zero start is the solution, so the solve ends before its first product."""
    import dataclasses
    s = dataclasses.replace(synth.tiny_cell(40, 16.0, 8, min_dist=1.2), grid=(20, 20, 20))
    ctx, t = amoeba.context_for(s, precision=prec, device=DEV)
    try:
        mu, ep, it, st = ctx.polarize(t["pos"], torch.zeros_like(t["pos"]), tol_debye=1e-8)
        assert st == amoeba.AMOEBA_OK and it == 0
        assert torch.count_nonzero(mu) == 0 and ep == 0.0
    finally:
        ctx.close()


def test_error_paths(c1):
    p = amoeba.Context(c1.n, c1.box, grid=c1.grid)
    pos = torch.tensor(c1.pos, device=DEV)
    with pytest.raises(amoeba.AmoebaError) as ei:
        p.build_blocklist(pos)  # parameters not set yet is allowed; perm field is not
        p.dipole_matvec(pos, torch.zeros_like(pos))
    assert ei.value.status == amoeba.AMOEBA_E_STATE
    p.close()
    ctx, t = amoeba.context_for(c1, precision="fp64", device=DEV)
    # stale list: buffer 0, any motion invalidates it
    moved = t["pos"] + 0.01
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.dipole_matvec(moved, torch.zeros_like(moved))
    assert ei.value.status == amoeba.AMOEBA_E_LIST
    # NaN in a dipole
    bad = torch.zeros_like(t["pos"])
    bad[5, 1] = float("nan")
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.dipole_matvec(t["pos"], bad)
    assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
    # non-convergence returns the last iterate
    e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
    mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-12, max_iter=3)
    assert st == amoeba.AMOEBA_NOT_CONVERGED and it == 3 and torch.isfinite(mu).all()
    mu0, _, it0, st0 = ctx.polarize(t["pos"], e, tol_debye=1e-5, max_iter=0)
    assert st0 == amoeba.AMOEBA_NOT_CONVERGED and it0 == 0 and torch.count_nonzero(mu0) == 0
    # NaN in the permanent field or in a given guess: reported, and the next solve is unaffected
    ebad = e.clone()
    ebad[7, 2] = float("inf")
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.polarize(t["pos"], ebad, tol_debye=1e-5)
    assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.polarize(t["pos"], e, mu_guess=bad, tol_debye=1e-5)
    assert ei.value.status == amoeba.AMOEBA_E_NUMERIC
    mu_a, ep_a, it_a, st_a = ctx.polarize(t["pos"], e, tol_debye=1e-8)
    mu_b, ep_b, it_b, st_b = ctx.polarize(t["pos"], e, mu_guess=mu_a, tol_debye=1e-7)
    assert st_a == st_b == amoeba.AMOEBA_OK and it_b == 0 and ep_b == ep_a
    assert torch.equal(mu_a, mu_b)
    # a quadrupole with a trace is rejected
    qbad = t["quad"].clone()
    qbad[4, 0] += 1e-6
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.perm_field(t["pos"], t["q"], t["dip"], qbad)
    assert ei.value.status == amoeba.AMOEBA_E_INVALID
    # FP64 mode sums with FP64 atomics (order-dependent rounding): equal to rounding, not bitwise
    assert torch.allclose(ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"]), e, rtol=1e-13, atol=1e-16)
    # invalid CSR: one direction missing
    sc_j = t["sc_j"].clone()
    sc_j[0] = (sc_j[0] + 7) % c1.n
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.set_atoms(t["alpha"], t["thole"], t["sc_ptr"], sc_j, t["sc_s"])
    assert ei.value.status == amoeba.AMOEBA_E_INVALID
    neg = t["alpha"].clone()
    neg[3] = -1.0
    with pytest.raises(amoeba.AmoebaError) as ei:
        ctx.set_atoms(neg, t["thole"], t["sc_ptr"], t["sc_j"], t["sc_s"])
    assert ei.value.status == amoeba.AMOEBA_E_INVALID
    ctx.close()


def test_range_and_workspace_errors(c1):
    """Mixed precision keeps fields as fixed-point integers held in FP64, exact below 8192 e/A^2:
    the permanent field, the product and the solve report AMOEBA_E_OVERFLOW beyond that range
    (charges, dipoles or the permanent field scaled up until the host-read check trips), and the
    context stays usable.  A workspace cap below what a context needs is AMOEBA_E_NOMEM."""
    print("[gpu] range and workspace errors", flush=True)
    ctx, t = amoeba.context_for(c1, precision="mixed", device=DEV)
    try:
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.perm_field(t["pos"], t["q"] * 1e6, t["dip"], t["quad"])
        assert ei.value.status == amoeba.AMOEBA_E_OVERFLOW
        e = ctx.perm_field(t["pos"], t["q"], t["dip"], t["quad"])
        assert float(e.abs().max()) < 100.0
        with pytest.raises(amoeba.AmoebaError) as ei:
            ctx.dipole_matvec(t["pos"], torch.full_like(t["pos"], 1e6))
        assert ei.value.status == amoeba.AMOEBA_E_OVERFLOW
        with pytest.raises(amoeba.AmoebaError) as ei:
            # the tolerance scales with the field, so that the solve converges and its accepted
            # dipoles reach the range check
            ctx.polarize(t["pos"], e * 1e5, tol_debye=1.0, max_iter=100)
        assert ei.value.status == amoeba.AMOEBA_E_OVERFLOW
        mu, ep, it, st = ctx.polarize(t["pos"], e, tol_debye=1e-5, max_iter=100)
        assert st == amoeba.AMOEBA_OK and torch.isfinite(mu).all()
    finally:
        ctx.close()
    with pytest.raises(amoeba.AmoebaError) as ei:
        amoeba.Context(c1.n, c1.box, grid=c1.grid, precision="mixed", max_workspace_bytes=1 << 16)
    assert ei.value.status == amoeba.AMOEBA_E_NOMEM
